#!/usr/bin/env python
"""Faces meshed per second by analytic marching on one MI355X.

One step is one pass of the whole hot path over one shape: dichotomy seeding
of 1,024 rays, marching every reachable analytic cell (chain, clip, vertex
solves, neighbour flips, hash deduplication) and emitting the CSR mesh.  The
network weights and the rays are resident in HBM before the timed region.

Workload of `value`: a 3->[90]x6->1 ReLU MLP fitted to the signed distance of
a union of 8 random spheres (frozen fixture am_workloads/data/c2.npz), seeded
by 128 Fibonacci directions from each sphere centre; it stands in for the
paper's D6-W60 ShapeNet fits (Table 4).  The other forms (split-BF16 on the
same net; plain and split-BF16 on the 3->[256]x8->1 superquadric fit) are
timed the same way and reported under "forms".

The timed plain steps are device-driven (each step reads its frontier on the
device; the host reads the counters once per 8 steps) and launched one by
one so that HIP events time every kernel class.  Host-driven steps and HIP
graph replays of the same steps are reported as forms.

Prints one JSON line with the metric, a roofline entry for the dominant
kernel (its average duration from HIP events recorded on the library's
stream during the timed steps) and the CPU oracle's rate on a bounded sample
of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "faces meshed/sec on 1 MI355X (plain vs learned+BF16 form); exact cell-set match"
PEAK_FP64_MFMA_TFLOPS = 78.6
PEAK_BF16_MFMA_TFLOPS = 2500.0
PEAK_HBM_GBS = 8000.0
# measured HBM traffic of kernels, written from rocprofv3 --pmc runs (profile_summary.py traffic)
PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2106_10031_amd", "csrc", f)
                  for f in ("am_kernels.hip", "am_internal.h")]


def workload(name: str):
    from am_workloads import nets, seeds
    if name in ("c2", "c3", "c5"):
        net = nets.load_fitted(name)
        prim = np.load(os.path.join(nets.DATA_DIR, f"{name}_primitives.npz"))
        o, d = seeds.centre_rays(prim["p0"], 128)
        desc = {"c2": "3->[90]x6->1 ReLU SDF fit of 8 random spheres (FP32 weights, FP64 geometry), 1024 dichotomy rays",
                "c3": "3->[256]x8->1 ReLU SDF fit of 8 random superquadrics (FP32 weights), 1024 dichotomy rays",
                "c5": "3->[512]x8->1 ReLU SDF fit of 8 random spheres (FP32 weights), 1024 dichotomy rays"}[name]
        return net, o, d, desc
    if name == "c1":
        net = nets.c1_net()
        o, d = seeds.axis_ray()
        return net, o, d, "0.1*MLP(3->64->64->1)+max-norm-0.5 (FP64), one ray along +x"
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


def sample_codes(codes_dev, k: int = 20000, seed: int = 3) -> np.ndarray:
    """A random sample of k face codes (all of them if fewer), as host uint64."""
    import torch
    F = codes_dev.shape[0]
    if F <= k:
        return codes_dev.cpu().numpy().view(np.uint64)
    g = torch.Generator(device="cpu").manual_seed(seed)
    idx = torch.randperm(F, generator=g)[:k].to(codes_dev.device)
    return codes_dev[idx].cpu().numpy().view(np.uint64)


def bf16_issued_flops_per_cell(net) -> float:
    """MFMA FLOPs the split-BF16 chain issues per cell: six BF16 products per
    block (l <- j), j >= 1, over 16-row output tiles and 32-wide K-steps, four
    columns."""
    r16 = lambda n: -(-n // 16) * 16
    r32 = lambda n: -(-n // 32) * 32
    return float(sum(6 * 2 * 4 * r16(net.widths[d]) * r32(net.widths[s]) for d, s, _ in net.blocks if s >= 1))


def form_fractions(net, r, precision, codes_sample):
    """Achieved rates of a form's chain kernel from its HIP-event times (host-
    driven steps): algorithmic FLOPs (active inputs only, FP64-equivalent) per
    second against the matrix peak of the chain's type (FP64 MFMA, or BF16
    MFMA for the split form, where the issued BF16 FLOPs are given too), and
    the rows it writes plus the codes it reads per second against HBM."""
    k = r["kernels"]
    if k["chain_launches"] <= 0 or k["chain_ms"] <= 0:
        return None
    cells = r["stats"]["cells"] * r["steps"]
    t = k["chain_ms"] * 1e-3
    alg = chain_flops_per_cell(net, codes_sample) * cells / t / 1e12
    N, M = net.n_hidden, net.n_heads
    W = max(1, -(-N // 64))
    row_bytes = (N + M) * 4 * (4 if precision else 8) + W * 8
    gbs = row_bytes * cells / t / 1e9
    e = {"chain_ms_per_step": round(k["chain_ms"] / r["steps"], 3),
         "chain_algorithmic_tflops": round(alg, 3),
         "mfma_peak_tflops": PEAK_BF16_MFMA_TFLOPS if precision else PEAK_FP64_MFMA_TFLOPS,
         "mfma_frac": round(alg / (PEAK_BF16_MFMA_TFLOPS if precision else PEAK_FP64_MFMA_TFLOPS), 6),
         "chain_hbm_gbs": round(gbs, 1), "hbm_frac": round(gbs / PEAK_HBM_GBS, 5)}
    if precision:
        iss = bf16_issued_flops_per_cell(net) * cells / t / 1e12
        e["chain_bf16_issued_tflops"] = round(iss, 2)
        e["mfma_frac_issued"] = round(iss / PEAK_BF16_MFMA_TFLOPS, 5)
    return e


def kernel_source_digest() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per launch of a kernel on the 6x90 fit from the committed
    counter runs (profiles/traffic_*.json, written by profile_summary.py
    traffic), or None when none was taken on this kernel or the kernel
    sources changed since."""
    import glob
    for path in sorted(glob.glob(os.path.join(PROFILES, "traffic_*.json"))):
        try:
            t = json.load(open(path))
        except (OSError, ValueError):
            continue
        if t.get("kernel", "").replace("am::", "") != kernel:
            continue
        if t.get("kernel_source_digest") != kernel_source_digest():
            return None
        return t
    return None


def host_cpu():
    """Model name and logical CPU counts of the host (from /proc/cpuinfo)."""
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
    return {"model": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def cpu_baseline(net, o, d, budget_s: float):
    """The oracle as it stands on the host cores: the single-threaded build on
    a BFS prefix of the workload, and the batched march (the same per-cell
    routines, each batch of active cells spread over OpenMP threads) on as
    much of the march as fits the budget."""
    from oracle import oracle as O
    on = O.OracleNet(net)
    t0 = time.perf_counter()
    codes, ams, _, _ = on.seed_rays(o, d)
    t_seed = time.perf_counter() - t0
    t1 = time.perf_counter()
    probe = on.march(codes, ams, max_cells=20000)
    per_cell = (time.perf_counter() - t1) / max(1, probe.stats["cells"])
    # later cells cost more than the first ones (larger tables), hence the 0.4
    half = 0.5 * budget_s
    cells = int(max(20000, min(2_000_000, 0.4 * half / max(per_cell, 1e-7))))
    t2 = time.perf_counter()
    mesh = on.march(codes, ams, max_cells=cells)
    t_march = time.perf_counter() - t2
    faces = mesh.n_faces
    rate1 = faces / (t_seed + t_march)
    single = {"value": round(rate1, 1), "unit": "faces/s", "cores": 1,
              "sample": f"dichotomy seeding of {len(o)} rays ({t_seed:.2f} s) + FIFO march of the first "
                        f"{min(cells, mesh.stats['cells'])} cells ({faces} faces, {t_march:.2f} s), "
                        f"single-threaded C oracle (gcc -O2), FP64"}
    om = O.OracleNet(net, lib_path=O.OMP_LIB_PATH)
    threads = om.threads()
    cells_p = int(max(20000, min(50_000_000, 0.4 * half * threads / max(per_cell, 1e-7))))
    t3 = time.perf_counter()
    mesh_p = om.march(codes, ams, max_cells=cells_p, batch=16384)
    t_par = time.perf_counter() - t3
    full = mesh_p.stats["cells"] < cells_p
    rate_p = mesh_p.n_faces / (t_seed + t_par)
    return {"value": round(rate_p, 1), "unit": "faces/s", "cores": threads, "kind": "oracle",
            "sample": f"dichotomy seeding of {len(o)} rays ({t_seed:.2f} s, one thread) + "
                      + ("the whole march" if full else f"FIFO march of the first {cells_p} cells")
                      + f" ({mesh_p.n_faces} faces, {t_par:.2f} s) with faces of each batch of 16384 active cells "
                        f"on {threads} OpenMP threads (gcc -O3, no contraction), C oracle, FP64",
            "single_thread": single, "host": host_cpu()}


def train_scorer(B, dev, max_cells):
    """Trains the proposal scorer on the GPU on rows the clip writes while
    marching the C1 net, the 6x90 fit and the 8x256 fit (at most 2^20 rows
    each); returns (params, info)."""
    import torch
    from am_workloads import seeds
    from paper_2106_10031_amd import learn
    t0 = time.perf_counter()
    Xs, ys = [], []
    for name in ("c1", "c2", "c3"):
        net, o, d, _ = workload(name)
        if name == "c1":
            o, d = seeds.random_rays(64, seed=11)
        ctx = B.Context(0).load_net(net)
        X, y = learn.collect(ctx, torch.as_tensor(o, device=dev), torch.as_tensor(d, device=dev), cap=1 << 20,
                             max_cells=max_cells)
        Xs.append(X.clone())
        ys.append(y.clone())
        ctx.close()
    X, y = torch.cat(Xs), torch.cat(ys)
    t1 = time.perf_counter()
    ctx = B.Context(0)
    params, losses = learn.train(ctx, X, y, steps=150, lr=3e-3)
    ctx.close()
    t2 = time.perf_counter()
    return params, {"rows": int(X.shape[0]), "positive_rate": round(float(y.float().mean()), 4),
                    "loss_first": round(losses[0], 4), "loss_last": round(losses[-1], 4),
                    "collect_s": round(t1 - t0, 2), "train_s": round(t2 - t1, 2),
                    "steps": 150, "scorer": "8 features (padded 32) -> 128 -> 128 -> 1, FP16 weights on MFMA"}


def cell_set_digest(out) -> str:
    """Order-independent 64-bit digest of a march's cell set (code words,
    argmax, shape id of every face), computed on the device: each face's
    words are mixed with fixed odd multipliers and the mixed values summed
    modulo 2^64.  Equal digests mean equal cell sets with overwhelming
    probability, whatever the discovery order."""
    import torch
    codes = out["codes"]
    F, W = codes.shape
    if F == 0:
        return "0" * 16
    g = torch.Generator(device="cpu").manual_seed(20210618)
    mult = torch.randint(1, 2 ** 62, (W + 2,), generator=g, dtype=torch.int64) * 2 + 1
    mult = mult.to(codes.device)
    h = (codes * mult[:W]).sum(dim=1)
    h = h + out["argmax"].to(torch.int64) * mult[W] + out["shape"].to(torch.int64) * mult[W + 1]
    h = h ^ (h >> 29)
    h = h * int(mult[0].item())
    h = h ^ (h >> 32)
    total = int(h.sum().item()) & (2 ** 64 - 1)
    return f"{total:016x}"


GOLDEN_DIR = os.path.join(ROOT, "tests", "golden")


def golden_check(ctx, name: str):
    """The context's last mesh against the oracle's record of the workload
    (tests/golden/<name>.json, written by the CPU oracle alone): faces and
    corners, and SHA-256 digests of the canonical cell set (codes, argmax),
    cycles (polygon sizes, edge ids) and adjacency (neighbour face per edge),
    all exact; sampled vertices within 1e-9 relative.  Outside the timed
    region.  None when there is no record."""
    import hashlib
    path = os.path.join(GOLDEN_DIR, f"{name}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    smp = np.load(os.path.join(GOLDEN_DIR, f"{name}_verts.npz"))
    out = ctx.fetch(sorted=True)
    off = out["offsets"].cpu().numpy()
    codes = out["codes"].cpu().numpy().view(np.uint64)
    am = out["argmax"].cpu().numpy()
    ids = out["ids"].cpu().numpy()
    nbr = out["nbr"].cpu().numpy()
    h1 = hashlib.sha256(np.ascontiguousarray(codes, "<u8").tobytes())
    h1.update(np.ascontiguousarray(am, "<i4").tobytes())
    h2 = hashlib.sha256(np.diff(off).astype("<i8").tobytes())
    h2.update(np.ascontiguousarray(ids, "<i4").tobytes())
    h3 = hashlib.sha256(np.ascontiguousarray(nbr, "<i8").tobytes())
    got = {"cell_set": h1.hexdigest(), "cycles": h2.hexdigest(), "adjacency": h3.hexdigest()}
    F = len(off) - 1
    match = (F == rec["faces"] and int(off[-1]) == rec["face_verts"]
             and all(got[k] == rec["sha256"][k] for k in got))
    verr = None
    if F == rec["faces"]:
        fs = smp["faces"]
        lo, hi = off[fs], off[fs + 1]
        idx = np.concatenate([np.arange(a, b) for a, b in zip(lo, hi)])
        if len(idx) == len(smp["verts"]):
            v = out["verts"][torch_index(idx, out["verts"].device)].cpu().numpy()
            ref = smp["verts"]
            verr = float((np.abs(v - ref).max(axis=1) / np.maximum(1.0, np.abs(ref).max(axis=1))).max())
        else:
            match = False
    match = match and verr is not None and verr <= 1e-9
    return {"golden_match": bool(match), "record": os.path.relpath(path, ROOT), "faces": F,
            "digests_equal": {k: got[k] == rec["sha256"][k] for k in got},
            "sampled_faces": int(len(smp["faces"])), "max_sampled_vertex_rel_err": verr}


def torch_index(idx, device):
    import torch
    return torch.as_tensor(idx, dtype=torch.int64, device=device)


def chain_kernel_name(net, groups, graph_steps):
    """The chain kernel the timed steps launch: device-driven steps take the
    variant of the 2^14-cell bucket (the gathered tile becomes the 4-cell
    one); host-driven steps mix buckets."""
    if graph_steps <= 0:
        return "k_chain_f64 (tile variants by launch size)"
    v = groups[2]
    wide = max(net.widths[1:-1]) > 128
    if v >= 6:
        mt = max((w + 15) // 16 for w in net.widths[1:])
        mtw = 2 if v == 8 else 1
        while mtw <= 4 and -(-mt // mtw) > (16 if mtw == 1 else 8):
            mtw *= 2
        f32 = all(np.array_equal(W.astype(np.float32).astype(np.float64), W) for _, _, W in net.blocks)
        return f"k_chain_lb<{2 if v == 7 else 1}, {mtw}, {'float' if f32 else 'double'}>"
    return {1: "k_chain_f64<1, 8>", 2: "k_chain_f64<2, 4>", 3: "k_chain_f64_res<8>" if wide else "k_chain_f64_lds<8>",
            4: "k_chain_f64<4, 4>", 5: "k_chain_f64<1, 8>"}[v]


def persist_kernel_name(net) -> str:
    """The persistent march kernel the library launches for `net`: for
    hidden layers of at most 256 units the ping-pong staged-B tile (2 with
    FP32 weight fragments when every weight is an FP32 number, else 1), else
    the dense tile (0)."""
    kpad = -(-max(net.widths[1:-1]) // 32) * 32
    if kpad > 256:
        return "k_march_persist<0>"
    f32 = all(np.array_equal(W.astype(np.float32).astype(np.float64), W) for _, _, W in net.blocks)
    return "k_march_persist<2>" if f32 else "k_march_persist<1>"


def time_form(ctx, o_d, d_d, precision, steps, warmup, max_cells, propose=0, tune=False, graph_steps=0,
              face_routine=0, time_kernels=None, kernel_path=0):
    """Times `steps` full passes (seed + march + fetch) after `warmup` passes
    (and, with tune, the chain-tile autotuner run on the warm-up's cells).
    Kernel-class durations come from HIP events recorded on the library's
    stream (host-driven steps only: graph replays are timed as a whole)."""
    import torch

    def step():
        ctx.seed_rays(o_d, d_d)
        tk = graph_steps == 0 if time_kernels is None else time_kernels
        st = ctx.march(max_cells=max_cells, time_kernels=tk, precision=precision, propose=propose,
                       graph_steps=graph_steps, face_routine=face_routine, kernel_path=kernel_path)
        out = ctx.fetch()
        return st, out

    for _ in range(max(1, warmup) if tune else warmup):
        step()
    if tune:
        ctx.tune_chain(reps=3)
        if warmup > 0:
            step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    out = None
    for _ in range(steps):
        st, out = step()
        stats.append(st)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    faces = stats[-1]["faces"]
    assert all(s["faces"] == faces for s in stats), "face count changed between steps"
    agg = {k: sum(s[k] for s in stats) for k in ("chain_ms", "clip_ms", "hash_ms", "march_ms",
                                               "chain_launches", "clip_launches")}
    return {"faces": faces, "ms_per_step": (t1 - t0) * 1e3 / steps, "faces_per_s": faces * steps / (t1 - t0),
            "stats": stats[-1], "kernels": agg, "out": out, "steps": steps}


def mesh_form(ctx, mesh, reps=5):
    """The welded output Z = {V, {P}} (Sec. 3) of a fetched march: shared
    vertices (am_weld) and fan triangles (am_triangles), timed together;
    then their simplification (am_simplify), timed alone."""
    import torch
    for rep in range(reps + 1):
        if rep == 1:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        cv, vx, unp = ctx.weld(mesh)
        tri = ctx.triangles(mesh["offsets"], cv)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    F = mesh["offsets"].shape[0] - 1
    out = {"ms": round(ms, 3), "faces": int(F), "corners": int(cv.shape[0]), "vertices": int(vx.shape[0]),
           "triangles": int(tri.shape[0]), "unpaired_edges": int(unp),
           "faces_per_s": round(F / (ms * 1e-3), 1) if ms > 0 else None}
    # quadric edge-collapse simplification (Sec. 4.4) of those triangles to 10 %
    target = int(tri.shape[0]) // 10
    for rep in range(3):
        if rep == 1:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        v2, t2, rounds, bad = ctx.simplify(vx, tri, target)
    torch.cuda.synchronize()
    out["simplify"] = {"ms": round((time.perf_counter() - t0) * 1e3 / 2, 3), "target_triangles": target,
                       "triangles": int(t2.shape[0]), "vertices": int(v2.shape[0]), "rounds": int(rounds)}
    return out


def seeding_forms(ctx, o, d, max_cells, reps=5):
    """Triggering (Sec. 4.3): dichotomy along the 1,024 rays against sphere
    tracing from their midpoints, each timed alone, and the faces marched
    from the sphere-tracing seeds."""
    import torch
    dev = ctx.device
    o_d = torch.as_tensor(o, dtype=torch.float64, device=dev)
    d_d = torch.as_tensor(d, dtype=torch.float64, device=dev)
    mid = (o_d + 0.5 * d_d).contiguous()
    out = {}
    for name in ("dichotomy", "sphere_tracing"):
        for rep in range(reps + 1):
            if rep == 1:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
            if name == "dichotomy":
                status = ctx.seed_rays(o_d, d_d)
            else:
                status, iters, _ = ctx.seed_points_st(mid)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / reps
        st = status.cpu().numpy()
        e = {"ms": round(ms, 3), "points": int(len(st)), "seeded": int((st == 0).sum())}
        if name == "sphere_tracing":
            it = iters.cpu().numpy()[st == 0]
            e["mean_steps"] = round(float(it.mean()), 2) if len(it) else None
            e["faces_marched_from_seeds"] = ctx.march(max_cells=max_cells)["faces"]
        out[name] = e
    return out


def ensemble_form(B, dev, steps):
    """Max-pooled ensemble of 4 depth-4 width-32 sub-networks (Sec. 5.2)."""
    import torch
    from am_workloads import nets, seeds
    net = nets.ensemble_net()
    cs = np.array([c for c, r in nets.ensemble_centres()])
    o, d = seeds.centre_rays(cs, 32)
    ctx = B.Context(0).load_net(net)
    r = time_form(ctx, torch.as_tensor(o, device=dev), torch.as_tensor(d, device=dev), 0, steps, 1, 1 << 21,
                  tune=True)
    ctx.close()
    return {"faces_per_s": round(r["faces_per_s"], 1), "ms_per_step": round(r["ms_per_step"], 3),
            "faces": r["faces"],
            "workload": "max over 4 logits r_i - |x - c_i|_1 - 0.3 MLP_i(x - c_i), MLP_i 4 x 32 ReLU "
                        "(untrained), 128 rays from the centres"}


def c4_forms(B, dev, steps, max_cells, scorer=None, graph_steps=8):
    """The 64-shape decoder batch: one batched march (all shapes in one
    frontier, chain tiles autotuned on it; device-driven steps replayed from
    a captured graph) against one march per shape; with a scorer, also the
    batched march with the split-BF16 chain and learned proposals together,
    replayed the same way and checked against the plain batched cell set.
    The chain's MFMA and HBM fractions of both come from one more march each
    with host-driven steps and HIP events around every kernel class."""
    import torch
    from am_workloads import nets, seeds
    sb = nets.c4_batch()
    S = sb.n_shapes
    o_np, d_np, sh_np = nets.c4_seed_rays(S)
    o = torch.as_tensor(o_np, device=dev)
    d = torch.as_tensor(d_np, device=dev)
    sh = torch.as_tensor(sh_np, device=dev)
    ctx = B.Context(0).load_net(sb.net, shape_bias=sb.shape_bias)

    def march(**kw):
        ctx.seed_rays(o, d, shape_id=sh)
        return ctx.march(max_cells=max_cells, **kw)

    def timed(reps, **kw):
        march(**kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            st_ = march(**kw)
        torch.cuda.synchronize()
        return st_, (time.perf_counter() - t0) / reps

    march(time_kernels=True)
    groups, _ = ctx.tune_chain(reps=3)
    st_p, t_p = timed(steps, kernel_path=3)
    pers_digest = cell_set_digest(ctx.fetch())
    st, t_b = timed(steps, graph_steps=graph_steps)
    plain_out = ctx.fetch()
    counts = np.bincount(plain_out["shape"].cpu().numpy(), minlength=S)
    plain_digest = cell_set_digest(plain_out)
    codes_s = sample_codes(plain_out["codes"])
    plain_verts = ctx.fetch(sorted=True)["verts"] if scorer is not None else None
    st_k = march(time_kernels=True)      # host-driven, HIP events: the chain's fractions
    fr_plain = form_fractions(sb.net, {"kernels": st_k, "stats": st_k, "steps": 1}, 0, codes_s)
    combined = None
    if scorer is not None:
        ctx.prop_set(scorer, k=16, rho=6.0)
        st_c, t_c = timed(steps, graph_steps=graph_steps, precision=1, propose=1)
        assert st_c["faces"] == st["faces"], "learned + split-BF16 batched march changed the face count"
        dg = cell_set_digest(ctx.fetch())
        gv = ctx.fetch(sorted=True)["verts"]
        verr = ((gv - plain_verts).abs().amax(dim=1) / plain_verts.abs().amax(dim=1).clamp(min=1.0)).max()
        st_ck = march(time_kernels=True, precision=1, propose=1)
        fr_c = form_fractions(sb.net, {"kernels": st_ck, "stats": st_ck, "steps": 1}, 1, codes_s)
        combined = {"faces_per_s": round(st_c["faces"] / t_c, 1), "ms_per_step": round(t_c * 1e3, 3),
                    "faces": st_c["faces"], "cell_set_digest": dg, "exact_cell_set_match": dg == plain_digest,
                    "vs_plain_batched": round(t_b / t_c, 4),
                    "launch": f"device-driven steps, {graph_steps} per HIP graph replay",
                    "precision": "split-BF16 chain (3 terms, 6 MFMA products, FP32 accumulate); FP64 clip and "
                                 "vertex solves; uncertified cells redone in FP64",
                    "proposals": "top-16 lines by the trained scorer clipped before the every-line pass",
                    "vertex_tol": 1e-5,
                    "split_row_eps": st_c["split_row_eps"], "split_margin": st_c["split_margin"],
                    "certificate_measured_on_vertices": st_c["calib_vertices"],
                    "max_vertex_rel_err_vs_fp64": float(verr.item()),
                    "escalated_cells": st_c["escalated"],
                    "escalated_fraction": round(st_c["escalated"] / max(1, st_c["cells"]), 4),
                    "accept_rate": round(st_c["prop_accepted"] / max(1, st_c["prop_cells"]), 4),
                    "chain_roofline": fr_c}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    faces_single = 0
    for s in range(S):
        m = sh_np == s
        ctx.seed_rays(o[m], d[m], shape_id=sh[m])
        faces_single += ctx.march(max_cells=max_cells)["faces"]
    torch.cuda.synchronize()
    t_s = time.perf_counter() - t0
    assert faces_single == st["faces"], "batched and per-shape marches differ"
    ctx.close()
    desc = ("64 shapes of one decoder [x; z] (3+256) -> [512]x8 -> 1 with [x; z] re-entering layer 4, "
            "trained as an auto-decoder on unions of 1-8 spheres at log-uniform scales 0.03..0.6; shape s "
            "marched in a box of half-size 1.2e-3..0.125 (log-spaced) centred on its surface, one seed ray each")
    out = {"c4_batched": {"faces_per_s": round(st["faces"] / t_b, 1), "ms_per_step": round(t_b * 1e3, 3),
                           "faces": st["faces"], "march_steps": st["steps"], "cell_set_digest": plain_digest,
                           "launch": f"device-driven steps, {graph_steps} per HIP graph replay",
                           "faces_per_shape_min_max": [int(counts.min()), int(counts.max())],
                           "chain_groups_tuned": groups, "workload": desc, "chain_roofline": fr_plain},
            "c4_per_shape": {"faces_per_s": round(faces_single / t_s, 1), "ms_per_step": round(t_s * 1e3, 3),
                             "faces": faces_single, "note": "one march per shape, same context, one pass"},
            "c4_batched_persistent": {"faces_per_s": round(st_p["faces"] / t_p, 1),
                                      "ms_per_step": round(t_p * 1e3, 3), "faces": st_p["faces"],
                                      "cell_set_digest": pers_digest,
                                      "exact_cell_set_match": pers_digest == plain_digest,
                                      "launch": "one persistent launch for all 64 shapes"}}
    if combined is not None:
        out["c4_learned_bf16"] = combined
    return out


def chain_sweep(B, name, counts, groups, reps=10):
    """The affine chain alone (am_chain) at several cell counts per launch.
    Codes are random (each unit on with probability 1/2), not cells of the
    surface: the dense chain does the same work for any code.  Times are
    HIP events around each call, so they include the unpadding copy;
    a kernel trace of the same run gives the chain kernel by itself."""
    import torch
    net = workload(name)[0]
    ctx = B.Context(0).load_net(net)
    if groups:
        ctx.set_chain_groups(groups)
    rng = np.random.default_rng(1)
    out = []
    for n in counts:
        codes = torch.as_tensor(rng.integers(0, 2 ** 62, size=(n, ctx.W), dtype=np.int64), device="cuda")
        ctx.chain(codes)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(ctx.stream)
        for _ in range(reps):
            ctx.chain(codes)
        e1.record(ctx.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out.append({"cells": n, "ms_per_call": round(ms, 4), "ns_per_cell": round(ms * 1e6 / n, 2)})
        print(f"[bench] chain sweep {name} {n} cells: {ms * 1e3:.1f} us per call", file=sys.stderr, flush=True)
    return {"chain_sweep": name, "chain_groups": ctx.chain_groups(), "calls": out}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c5"])
    ap.add_argument("--max-cells", type=int, default=1 << 24)
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms",
                    default="seeding,mesh,pivot,bf16,distance,learned,learned_bf16,c3,c3_bf16,c3_learned_bf16,"
                            "ensemble,c4,c4_learned_bf16,c5,c5_learned_bf16",
                    help="other forms to time on the same net (seeding, mesh, pivot, bf16, distance, learned, "
                         "learned_bf16), on "
                         "the 8x256 fit (c3, c3_bf16, c3_learned, c3_learned_bf16) and the 64-shape decoder "
                         "batch (c4; c4_learned_bf16: with the split-BF16 chain and learned proposals "
                         "together); empty for none")
    ap.add_argument("--graph-steps", type=int, default=8,
                    help="device-driven marching steps per counter read for the plain form (also timed as "
                         "graph replays); 0: host-driven steps")
    ap.add_argument("--chain-groups", default="",
                    help="fixed chain tile variants per launch-size bucket, e.g. 1,3,3,3 (default: autotune)")
    ap.add_argument("--legs", default="persistent,timed,graph,host",
                    help="legs of the plain form: persistent (the whole march as one persistent launch, HIP events "
                         "around it), timed (device-driven steps, HIP events around every kernel class), graph "
                         "(the same steps as graph replays), host (host-driven steps); value is the faster of "
                         "persistent and graph (else timed)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after the bench, copy this many MiB device-to-device (counter calibration)")
    ap.add_argument("--chain-sweep", default="",
                    help="instead of the bench: the workload's chain alone (am_chain) at these cell counts, "
                         "e.g. 256,1024,3500,14000, ten launches each (for a kernel trace)")
    a = ap.parse_args(argv)

    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the marching path runs on a single MI355X "
              "(multi-GPU sharding is described in the design notes, not built).", file=sys.stderr)
        return 2

    import torch
    from paper_2106_10031_amd import binding as B

    dev = torch.device("cuda", 0)
    if a.chain_sweep:
        print(json.dumps(chain_sweep(B, a.workload, [int(x) for x in a.chain_sweep.split(",")],
                                     [int(x) for x in a.chain_groups.split(",")] if a.chain_groups else None)))
        return 0
    forms_req = [f for f in a.forms.split(",") if f]

    def prepare(name):
        net, o, d, desc = workload(name)
        ctx = B.Context(0).load_net(net)
        o_d = torch.as_tensor(o, dtype=torch.float64, device=dev)
        d_d = torch.as_tensor(d, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        return net, o, d, desc, ctx, o_d, d_d

    learned_forms = [f for f in forms_req if "learned" in f]
    scorer, train_info = (train_scorer(B, dev, a.max_cells) if learned_forms else (None, None))
    if scorer is not None:
        print(f"[bench] scorer trained: {train_info}", file=sys.stderr, flush=True)

    net, o, d, desc, ctx, o_d, d_d = prepare(a.workload)
    if scorer is not None:
        ctx.prop_set(scorer, k=16, rho=6.0)
    # value: the faster launch of the plain form, the persistent march or
    # device-driven steps replayed from a captured HIP graph
    gs = a.graph_steps
    legs = set(x for x in a.legs.split(",") if x)
    fixed_groups = [int(x) for x in a.chain_groups.split(",")] if a.chain_groups else None
    if fixed_groups:
        ctx.set_chain_groups(fixed_groups)
    fp64_desc = "FP64 chain (MFMA), FP64 clip and vertex solves"
    forms = {}
    golden = {}
    runs = []   # (run, launch description, golden record check) of the legs that can give value
    # the whole march as one persistent launch (HIP events around it)
    pers = None
    pers_launch = ("one persistent launch: workgroups take discovered cells from a device-side queue, chain, "
                   "clip and insert their neighbours until none is left or in flight")
    if "persistent" in legs:
        pers = time_form(ctx, o_d, d_d, 0, a.steps, a.warmup, a.max_cells, kernel_path=3, time_kernels=True)
        gp = golden_check(ctx, a.workload)   # the last march is this configuration
        print(f"[bench] {a.workload} persistent: {pers['faces']} faces, {pers['ms_per_step']:.2f} ms/step, "
              f"golden {gp}", file=sys.stderr, flush=True)
        forms[f"{a.workload}_plain_persistent"] = {
            "faces_per_s": round(pers["faces_per_s"], 1), "ms_per_step": round(pers["ms_per_step"], 3),
            "precision": fp64_desc, "launch": pers_launch, "cell_set_digest": cell_set_digest(pers["out"])}
        runs.append((pers, pers_launch, gp))
    # device-driven steps (each step reads its frontier on the device; the
    # host reads the counters once per graph_steps steps), launched one by
    # one with HIP events around every kernel class (gives the stepped
    # kernels' rooflines), and the same steps replayed from a captured HIP
    # graph; host-driven steps are timed as a form
    timed = None
    if legs & {"timed", "graph", "host"}:
        timed = time_form(ctx, o_d, d_d, 0, a.steps, a.warmup, a.max_cells, tune=fixed_groups is None,
                          graph_steps=gs, time_kernels=True)
        if gs > 0:
            timed_launch = (f"device-driven steps launched one by one, {gs} per counter read, HIP events around "
                            "every kernel class")
        else:
            timed_launch = "host-driven steps, HIP events around every kernel class"
        gt = golden_check(ctx, a.workload)
        forms[f"{a.workload}_plain_timed"] = {
            "faces_per_s": round(timed["faces_per_s"], 1), "ms_per_step": round(timed["ms_per_step"], 3),
            "precision": fp64_desc, "launch": timed_launch}
        print(f"[bench] {a.workload}_plain_timed: {timed['ms_per_step']:.2f} ms/step", file=sys.stderr, flush=True)
        if gs > 0 and "graph" in legs:
            g = time_form(ctx, o_d, d_d, 0, a.steps, a.warmup, a.max_cells, graph_steps=gs)
            assert g["faces"] == timed["faces"], "graph-launched form changed the face count"
            g_launch = f"device-driven steps, {gs} per HIP graph replay"
            gg = golden_check(ctx, a.workload)
            forms[f"{a.workload}_plain_graph"] = {
                "faces_per_s": round(g["faces_per_s"], 1), "ms_per_step": round(g["ms_per_step"], 3),
                "precision": fp64_desc, "launch": g_launch, "cell_set_digest": cell_set_digest(g["out"])}
            print(f"[bench] {a.workload}_plain_graph: {g['ms_per_step']:.2f} ms/step", file=sys.stderr, flush=True)
            runs.append((g, g_launch, gg))
        else:
            runs.append((timed, timed_launch, gt))
    chain_tiles = {a.workload: ctx.chain_groups()}
    assert runs, "no leg of the plain form ran"
    assert all(r[0]["faces"] == runs[0][0]["faces"] for r in runs), "the legs disagree on the face count"
    main_run, main_launch, golden[a.workload] = min(runs, key=lambda r: r[0]["ms_per_step"])
    print(f"[bench] {a.workload} plain: {main_run['faces']} faces, {main_run['ms_per_step']:.2f} ms/step "
          f"({main_launch})", file=sys.stderr, flush=True)
    plain_digest = cell_set_digest(main_run["out"])
    forms[f"{a.workload}_plain"] = {"faces_per_s": round(main_run["faces_per_s"], 1),
                                    "ms_per_step": round(main_run["ms_per_step"], 3),
                                    "precision": fp64_desc, "launch": main_launch, "cell_set_digest": plain_digest}
    if timed is not None and gs > 0 and "host" in legs:
        r = time_form(ctx, o_d, d_d, 0, a.steps, a.warmup, a.max_cells)
        assert r["faces"] == main_run["faces"], "host-driven form changed the face count"
        forms[f"{a.workload}_plain_host"] = {
            "faces_per_s": round(r["faces_per_s"], 1), "ms_per_step": round(r["ms_per_step"], 3),
            "precision": fp64_desc,
            "launch": "host-driven steps (one counter read per step), HIP events around every kernel class"}
        print(f"[bench] {a.workload}_plain_host: {r['ms_per_step']:.2f} ms/step", file=sys.stderr, flush=True)
    bf16_desc = ("split-BF16 chain (3 terms, 6 MFMA products, FP32 accumulate); FP64 clip and vertex solves on "
                 "the FP32 rows; cells whose combinatorics or vertices (1e-5) are not certified are redone in FP64")
    if "mesh" in forms_req:
        forms[f"{a.workload}_mesh"] = mesh_form(ctx, main_run["out"])
        print(f"[bench] mesh: {forms[a.workload + '_mesh']}", file=sys.stderr, flush=True)
    if "seeding" in forms_req:
        forms[f"{a.workload}_seeding"] = seeding_forms(ctx, o, d, a.max_cells)
        print(f"[bench] seeding: {forms[a.workload + '_seeding']}", file=sys.stderr, flush=True)
    variants = {"pivot": (0, 0, 1), "bf16": (1, 0, 0), "distance": (0, 2, 0), "learned": (0, 1, 0),
                "learned_bf16": (1, 1, 0)}
    prop_desc = {0: None, 1: "top-16 lines by the trained scorer clipped before the every-line pass",
                 2: "top-16 lines by distance to the entry edge clipped before the every-line pass"}

    def record(key, r, precision, propose, routine=0, ref_digest=None, net_=None):
        e = {"faces_per_s": round(r["faces_per_s"], 1), "ms_per_step": round(r["ms_per_step"], 3),
             "faces": r["faces"], "precision": bf16_desc if precision else "FP64 chain (MFMA), FP64 clip"}
        if net_ is not None and (propose == 0 or precision) and not routine:
            fr = form_fractions(net_, r, precision, sample_codes(r["out"]["codes"]))
            if fr:
                e["chain_roofline"] = fr
        d = cell_set_digest(r["out"])
        e["cell_set_digest"] = d
        if ref_digest is not None:
            e["exact_cell_set_match"] = d == ref_digest
        if routine:
            st = r["stats"]
            e["precision"] = "FP64 chain (MFMA), FP64 pivoting walk"
            e["face_routine"] = ("pivoting (Sec. 4.2.1): each face traced from its entry edge, one ratio test "
                                 "over every line per vertex; seeds and cells without a usable entry edge clipped")
            e["walked_cells"] = st["pivot_cells"]
            e["clipped_cells"] = st["pivot_fallback"]
            e["clip_ms_per_step"] = round(r["kernels"]["clip_ms"] / r["steps"], 3)
        if precision:
            st_ = r["stats"]
            e["escalated_cells"] = st_["escalated"]
            e["escalated_fraction"] = round(st_["escalated"] / max(1, st_["cells"]), 4)
            e["split_row_eps"] = st_["split_row_eps"]
            e["split_margin"] = st_["split_margin"]
        if propose:
            st = r["stats"]
            e["proposals"] = prop_desc[propose]
            e["accept_rate"] = round(st["prop_accepted"] / max(1, st["prop_cells"]), 4)
            e["cuts_per_cell_in_check_pass"] = round(st["prop_cuts"] / max(1, st["prop_cells"]), 3)
        forms[key] = e
        print(f"[bench] {key}: {r['ms_per_step']:.2f} ms/step", file=sys.stderr, flush=True)

    for v, (precision, propose, routine) in variants.items():
        if v not in forms_req:
            continue
        r = time_form(ctx, o_d, d_d, precision, a.steps, a.warmup, a.max_cells, propose=propose,
                      face_routine=routine)
        assert r["faces"] == main_run["faces"], f"{v} form changed the face count"
        record(f"{a.workload}_{v}", r, precision, propose, routine, ref_digest=plain_digest, net_=net)

    # roofline of the dominant kernel of the value's launch.  Persistent: the
    # one fused kernel (chain, clip, insertion); its dense contraction is the
    # FP64 chain on MFMA, so its algorithmic flops are the chain's.  Stepped:
    # the chain (FP64 MFMA) or the clip (HBM: it reads every row the chain
    # wrote), whichever took longer.
    flops_cell = chain_flops_per_cell(net, sample_codes(main_run["out"]["codes"]))
    pers_entry = chain_entry = clip_entry = None
    if pers is not None:
        kp = pers["kernels"]
        p_ms = kp["chain_ms"] / max(1, kp["chain_launches"])   # the march's one launch
        p_cells = pers["stats"]["cells"]
        p_tflops = flops_cell * p_cells / (p_ms * 1e-3) / 1e12 if p_ms > 0 else 0.0
        pname = persist_kernel_name(net)
        ptraffic = measured_traffic(pname)
        pers_entry = {"kernel": pname, "bound": "mfma", "achieved": round(p_tflops, 4),
                      "peak": PEAK_FP64_MFMA_TFLOPS, "unit": "TFLOP/s",
                      "frac": round(p_tflops / PEAK_FP64_MFMA_TFLOPS, 6),
                      "traffic": ptraffic["bytes_per_launch"] if ptraffic else None,
                      "algorithmic_flops_per_cell": round(flops_cell, 1), "cells_per_launch": p_cells,
                      "avg_launch_ms": round(p_ms, 4), "timed_on": pers_launch + "; HIP events around the launch",
                      "note": "fused chain + clip + neighbour insertion in one launch; the FP64 chain is its only "
                              "dense contraction"}
        if ptraffic:
            pers_entry["traffic_note"] = ptraffic.get("note", "")
    if timed is not None:
        kst = timed["kernels"]
        st_t = timed["stats"]
        cells = st_t["cells"]
        chain_avg_ms = kst["chain_ms"] / max(1, kst["chain_launches"])
        cells_per_launch = cells * a.steps / max(1, kst["chain_launches"])
        chain_tflops = flops_cell * cells_per_launch / (chain_avg_ms * 1e-3) / 1e12 if chain_avg_ms > 0 else 0.0
        kname = chain_kernel_name(net, chain_tiles[a.workload], gs)
        traffic = measured_traffic(kname)
        split = {k: round(kst[k] / a.steps, 3) for k in ("chain_ms", "clip_ms", "hash_ms", "march_ms")}
        chain_entry = {"kernel": kname, "bound": "mfma",
                       "achieved": round(chain_tflops, 4),
                       "peak": PEAK_FP64_MFMA_TFLOPS, "unit": "TFLOP/s",
                       "frac": round(chain_tflops / PEAK_FP64_MFMA_TFLOPS, 6),
                       "traffic": traffic["bytes_per_launch"] if traffic else None,
                       "algorithmic_flops_per_cell": round(flops_cell, 1),
                       "cells_per_launch": round(cells_per_launch, 1),
                       "avg_launch_ms": round(chain_avg_ms, 5), "timed_on": timed_launch,
                       "time_split_ms_per_step": split}
        if traffic:
            chain_entry["traffic_note"] = traffic.get("note", "")
        # clip: per cell it reads the cell's rows, code, argmax, hints and
        # fingerprint and writes its face (ids, vertices, neighbour slots,
        # size, flags) and one candidate per edge (parent, slot, unit,
        # fingerprint, hints, key)
        N, M = net.n_hidden, net.n_heads
        W = max(1, -(-N // 64))
        mbar = st_t["face_verts"] / max(1, st_t["faces"])
        clip_bytes_cell = (N + M) * 32 + W * 8 + 4 + 12 + 8 + mbar * (4 + 24 + 4) + 8 + mbar * 32
        clip_avg_ms = kst["clip_ms"] / max(1, kst["clip_launches"])
        clip_gbs = clip_bytes_cell * cells_per_launch / (clip_avg_ms * 1e-3) / 1e9 if clip_avg_ms > 0 else 0.0
        ctraffic = measured_traffic("k_clip<double>")
        clip_entry = {"kernel": "k_clip<double>", "bound": "hbm", "achieved": round(clip_gbs, 2),
                      "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(clip_gbs / PEAK_HBM_GBS, 6),
                      "traffic": ctraffic["bytes_per_launch"] if ctraffic else None,
                      "algorithmic_bytes_per_cell": round(clip_bytes_cell, 1),
                      "cells_per_launch": round(cells_per_launch, 1),
                      "avg_launch_ms": round(clip_avg_ms, 5), "timed_on": timed_launch,
                      "time_split_ms_per_step": split}
        if ctraffic:
            clip_entry["traffic_note"] = ctraffic.get("note", "")
    stepped = None
    if chain_entry is not None:
        stepped = clip_entry if kst["clip_ms"] > kst["chain_ms"] else chain_entry
    if main_run is pers:
        roofline, roofline_other = pers_entry, stepped
    else:
        roofline, roofline_other = stepped, pers_entry
    ctx.close()

    for name in ("c3", "c5"):
        todo = [(v, pv) for v, pv in [("plain", (0, 0, 0))] + list(variants.items())
                if (name if v == "plain" else f"{name}_{v}") in forms_req]
        if name == a.workload or not todo:
            continue
        net3, _, _, _, ctx3, o3, d3 = prepare(name)
        if scorer is not None:
            ctx3.prop_set(scorer, k=16, rho=6.0)
        steps3 = max(1, min(a.steps, 3 if name == "c3" else 1))
        base = None
        base_digest = None
        for i, (v, (precision, propose, routine)) in enumerate(todo):
            r = time_form(ctx3, o3, d3, precision, steps3, 1 if name == "c3" else 0,
                          a.max_cells if name == "c3" else max(a.max_cells, 1 << 26), propose=propose,
                          tune=(i == 0), face_routine=routine)
            chain_tiles[name] = ctx3.chain_groups()
            if base is None:
                base = r["faces"]
            assert r["faces"] == base, f"{name} {v} form changed the face count"
            record(f"{name}_{v}", r, precision, propose, routine, ref_digest=base_digest, net_=net3)
            if base_digest is None:
                base_digest = forms[f"{name}_{v}"]["cell_set_digest"]
                golden[name] = golden_check(ctx3, name)
                print(f"[bench] golden {name}: {golden[name]}", file=sys.stderr, flush=True)
        ctx3.close()
    if "ensemble" in forms_req:
        forms["ensemble_4x_d4w32"] = ensemble_form(B, dev, a.steps)
        print(f"[bench] ensemble: {forms['ensemble_4x_d4w32']['ms_per_step']:.2f} ms/step", file=sys.stderr,
              flush=True)
    if "c4" in forms_req or "c4_learned_bf16" in forms_req:
        forms.update(c4_forms(B, dev, max(1, min(a.steps, 2)), a.max_cells,
                              scorer if "c4_learned_bf16" in forms_req else None))
        print(f"[bench] c4: {forms['c4_batched']['ms_per_step']:.1f} ms batched, "
              f"{forms['c4_per_shape']['ms_per_step']:.1f} ms per-shape"
              + (f", {forms['c4_learned_bf16']['ms_per_step']:.1f} ms learned + split-BF16"
                 if "c4_learned_bf16" in forms else ""), file=sys.stderr, flush=True)
    if train_info:
        forms["scorer_training"] = train_info
    forms["chain_tiles_tuned"] = {k: v for k, v in chain_tiles.items()}

    st = main_run["stats"]
    res = {"metric": METRIC, "value": round(main_run["faces_per_s"], 1), "unit": "faces/s", "n_gpus": 1,
           "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(main_run["ms_per_step"], 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic (frozen fitted fixture, seeded rays)",
           "config": {"workload": desc, "form": "plain", "launch": main_launch, "faces": st["faces"],
                      "face_verts": st["face_verts"],
                      "triangles": st["triangles"], "cells": st["cells"], "march_steps": st["steps"],
                      "seeds": st["seed_cells"], "degenerate": st["degenerate"]},
           "forms": forms, "roofline": roofline, "roofline_other_kernel": roofline_other,
           "golden": {k: g for k, g in golden.items() if g is not None},
           "golden_match": bool(golden.get(a.workload)) and all(g["golden_match"] for g in golden.values()
                                                                 if g is not None),
           "golden_unrecorded": sorted(k for k, g in golden.items() if g is None),
           "exact_cell_set_match": all(v.get("exact_cell_set_match", True) for v in forms.values()
                                       if isinstance(v, dict))}
    if not a.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(net, o, d, a.cpu_budget)
    if a.calib_copy_mib > 0:
        n = a.calib_copy_mib * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
