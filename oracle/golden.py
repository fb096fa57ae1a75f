"""Writes the oracle's reference records of the measured workloads.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``): it calls the CPU
oracle and nothing else, and writes ``tests/golden/<name>.json`` plus a small
vertex sample ``tests/golden/<name>_verts.npz``.  The GPU tests and the
benchmark compare their meshes with these records, so every number the
benchmark reports for a workload is tied to the oracle's mesh of it.

A record holds, for the mesh the oracle reaches from the workload's seeds
(Algorithm 1 from the dichotomy seeds of Sec. 4.3.2, faces in canonical
order: code words, then argmax):

* the counts: faces, face vertices, cells discovered (faces and empty ones),
  degenerate cells, distinct seed cells;
* three SHA-256 digests of little-endian arrays in canonical order
  (``canonical_digests``):
    - ``cell_set``:   codes ``[F][W]`` u64, then argmax ``[F]`` i32;
    - ``cycles``:     polygon sizes ``[F]`` i64, then edge ids ``[V]`` i32;
    - ``adjacency``:  neighbour face index per edge ``[V]`` i64 (-1 box edge);
* the vertices of every k-th face (k = max(1, F // 4096)) for a 1e-9
  comparison (vertices are not expected to be bit-equal, Sec. 2.2 rounding).

Run:  python -m oracle.golden c1 c2 c3      (C3 takes about 20 minutes on 8
cores with the OpenMP build of the oracle).
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN_DIR = os.path.join(ROOT, "tests", "golden")
SAMPLE_FACES = 4096


def canonical_digests(codes, argmax, offsets, ids, nbr) -> dict:
    """SHA-256 digests of a mesh given in canonical face order."""
    codes = np.ascontiguousarray(codes, dtype="<u8")
    argmax = np.ascontiguousarray(argmax, dtype="<i4")
    offsets = np.asarray(offsets, dtype=np.int64)
    m = np.ascontiguousarray(np.diff(offsets), dtype="<i8")
    ids = np.ascontiguousarray(ids, dtype="<i4")
    nbr = np.ascontiguousarray(nbr, dtype="<i8")
    h_cells = hashlib.sha256()
    h_cells.update(codes.tobytes())
    h_cells.update(argmax.tobytes())
    h_cyc = hashlib.sha256()
    h_cyc.update(m.tobytes())
    h_cyc.update(ids.tobytes())
    return {"cell_set": h_cells.hexdigest(), "cycles": h_cyc.hexdigest(),
            "adjacency": hashlib.sha256(nbr.tobytes()).hexdigest()}


def workload(name: str):
    """(net, ray origins, ray directions, description) of a measured workload."""
    from am_workloads import nets, seeds
    if name == "c1":
        o, d = seeds.axis_ray()
        return nets.c1_net(), o, d, "0.1*MLP(3->64->64->1)+max-norm-0.5 (FP64), one ray along +x"
    net = nets.load_fitted(name)
    prim = np.load(os.path.join(nets.DATA_DIR, f"{name}_primitives.npz"))
    o, d = seeds.centre_rays(prim["p0"], 128)
    return net, o, d, f"fitted fixture {name}, 1024 dichotomy rays (128 Fibonacci directions per primitive centre)"


def make(name: str, batch: int = 16384) -> dict:
    from oracle import oracle as O
    net, o, d, desc = workload(name)
    on = O.OracleNet(net, lib_path=O.OMP_LIB_PATH)
    t0 = time.perf_counter()
    codes, ams, _, st = on.seed_rays(o, d)
    mesh = on.march(codes, ams, batch=batch)
    wall = time.perf_counter() - t0
    F = mesh.n_faces
    k = max(1, F // SAMPLE_FACES)
    sample = np.arange(0, F, k, dtype=np.int64)
    m = np.diff(mesh.offsets)
    vs = np.concatenate([mesh.verts[mesh.offsets[f]:mesh.offsets[f + 1]] for f in sample]) if F else np.zeros((0, 3))
    rec = {
        "workload": name,
        "description": desc,
        "rays": int(len(o)),
        "rays_with_seed": int((st == 0).sum()),
        "faces": int(F),
        "face_verts": int(mesh.stats["face_verts"]),
        "cells": int(mesh.stats["cells"]),
        "seed_cells": int(mesh.stats["seeds_in"] - mesh.stats["seed_dup"]),
        "degenerate": int(mesh.stats["degenerate"]),
        "sha256": canonical_digests(mesh.codes, mesh.argmax, mesh.offsets, mesh.ids, mesh.nbr),
        "vertex_sample_every": int(k),
        "vertex_sample_faces": int(len(sample)),
        "written_by": "python -m oracle.golden " + name,
        "oracle_threads": on.threads(),
        "oracle_wall_s": round(wall, 1),
    }
    os.makedirs(GOLDEN_DIR, exist_ok=True)
    np.savez_compressed(os.path.join(GOLDEN_DIR, f"{name}_verts.npz"), faces=sample, m=m[sample], verts=vs)
    with open(os.path.join(GOLDEN_DIR, f"{name}.json"), "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    return rec


if __name__ == "__main__":
    for nm in sys.argv[1:] or ["c1", "c2"]:
        r = make(nm)
        print(json.dumps({k: r[k] for k in ("workload", "faces", "face_verts", "cells", "oracle_wall_s")}),
              flush=True)
