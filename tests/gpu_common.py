"""Helpers for the GPU parity tests (device mesh -> host, mesh comparison)."""
import dataclasses
import os
import sys

import numpy as np

import meshcheck as MC


def say(*a):
    """Names the case about to run on the GPU (flushed, so a fault still shows it)."""
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@dataclasses.dataclass
class HostMesh:
    codes: np.ndarray
    argmax: np.ndarray
    offsets: np.ndarray
    ids: np.ndarray
    verts: np.ndarray
    nbr: np.ndarray

    @property
    def n_faces(self):
        return len(self.offsets) - 1

    def face(self, f):
        a, b = self.offsets[f], self.offsets[f + 1]
        return self.ids[a:b], self.verts[a:b], self.nbr[a:b]


def fetch_host(ctx):
    from paper_2106_10031_amd.binding import mesh_to_host
    h = mesh_to_host(ctx.fetch())
    return HostMesh(h["codes"], h["argmax"], h["offsets"], h["ids"], h["verts"], h["nbr"])


def compare_meshes(ref, got, vtol=1e-9):
    """Cell set, cycles and adjacency bit-exact; vertices within vtol relative."""
    R = MC.by_code(ref)
    G = MC.by_code(got)
    missing = set(R) - set(G)
    extra = set(G) - set(R)
    assert not missing and not extra, f"{len(missing)} faces missing, {len(extra)} extra (of {len(R)})"
    worst = 0.0
    for k, (ids, vs, nb) in R.items():
        gi, gv, gn = G[k]
        assert np.array_equal(gi, ids), (k, gi, ids)
        assert gn == nb, (k, gn, nb)
        err = np.max(np.abs(gv - vs)) / max(1.0, np.max(np.abs(vs)))
        worst = max(worst, float(err))
    assert worst <= vtol, worst
    return worst


def canonical_order(mesh):
    """(face order, corner order) that sort faces by (code words, argmax)."""
    codes = np.asarray(mesh.codes, np.uint64)
    am = np.asarray(mesh.argmax)
    keys = [am] + [codes[:, w] for w in range(codes.shape[1] - 1, -1, -1)]
    order = np.lexsort(keys)
    off = np.asarray(mesh.offsets, np.int64)
    ms = np.diff(off)[order]
    starts = off[:-1][order]
    rel = np.arange(ms.sum()) - np.repeat(np.cumsum(ms) - ms, ms)
    return order, np.repeat(starts, ms) + rel


def canonical(mesh):
    """Faces sorted by (code words, argmax); neighbour indices remapped.

    Returns (codes, argmax, m, ids, verts, nbr) with the per-edge arrays
    concatenated in sorted face order.  Vectorised, for meshes with millions
    of faces.
    """
    codes = np.asarray(mesh.codes, np.uint64)
    am = np.asarray(mesh.argmax)
    order, idx = canonical_order(mesh)
    inv = np.empty_like(order)
    inv[order] = np.arange(len(order))
    ms = np.diff(np.asarray(mesh.offsets, np.int64))[order]
    nbr = np.asarray(mesh.nbr, np.int64)[idx]
    nbr = np.where(nbr >= 0, inv[np.maximum(nbr, 0)], nbr)
    return codes[order], am[order], ms, np.asarray(mesh.ids)[idx], np.asarray(mesh.verts)[idx], nbr


def compare_meshes_fast(ref, got, vtol=1e-9):
    """compare_meshes for large meshes: same bar, vectorised."""
    rc, ra, rm, ri, rv, rn = canonical(ref)
    gc, ga, gm, gi, gv, gn = canonical(got)
    assert rc.shape == gc.shape, (rc.shape, gc.shape)
    assert np.array_equal(rc, gc) and np.array_equal(ra, ga), "face sets differ"
    assert np.array_equal(rm, gm), "polygon sizes differ"
    assert np.array_equal(ri, gi), "edge id cycles differ"
    assert np.array_equal(rn, gn), "adjacency differs"
    scale = np.maximum(1.0, np.repeat(np.abs(rv).reshape(-1, 3).max(axis=1), 1))
    err = np.abs(gv - rv).max(axis=1) / np.maximum(1.0, np.abs(rv).max(axis=1))
    worst = float(err.max()) if len(err) else 0.0
    assert worst <= vtol, worst
    return worst


# ---------------------------------------------------------------- golden records
GOLDEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name):
    """The oracle's record of a workload (tests/golden/<name>.json and its
    vertex sample), or None when it has not been written."""
    import json
    p = os.path.join(GOLDEN_DIR, f"{name}.json")
    if not os.path.exists(p):
        return None
    rec = json.load(open(p))
    rec["sample"] = dict(np.load(os.path.join(GOLDEN_DIR, f"{name}_verts.npz")))
    return rec


def mesh_digests(codes, argmax, offsets, ids, nbr):
    """SHA-256 of the canonical arrays: codes then argmax; polygon sizes then
    edge ids; neighbour face per edge (little-endian, as the records hold)."""
    import hashlib
    m = np.diff(np.asarray(offsets, np.int64)).astype("<i8")
    a = hashlib.sha256(np.ascontiguousarray(codes, "<u8").tobytes())
    a.update(np.ascontiguousarray(argmax, "<i4").tobytes())
    b = hashlib.sha256(m.tobytes())
    b.update(np.ascontiguousarray(ids, "<i4").tobytes())
    c = hashlib.sha256(np.ascontiguousarray(nbr, "<i8").tobytes())
    return {"cell_set": a.hexdigest(), "cycles": b.hexdigest(), "adjacency": c.hexdigest()}


def check_golden(ctx, rec, vtol=1e-9):
    """The context's last mesh, fetched in canonical order, against an oracle
    record: counts and the three digests exact, sampled vertices within vtol
    relative.  Returns the worst sampled vertex error."""
    from paper_2106_10031_amd.binding import mesh_to_host
    h = mesh_to_host(ctx.fetch(sorted=True))
    F = len(h["offsets"]) - 1
    assert F == rec["faces"], (F, rec["faces"])
    assert int(h["offsets"][-1]) == rec["face_verts"], (int(h["offsets"][-1]), rec["face_verts"])
    assert np.all(h["shape"] == 0)
    dg = mesh_digests(h["codes"], h["argmax"], h["offsets"], h["ids"], h["nbr"])
    for k in ("cell_set", "cycles", "adjacency"):
        assert dg[k] == rec["sha256"][k], f"{rec['workload']}: {k} digest differs from the oracle's"
    s = rec["sample"]
    off = h["offsets"]
    got = np.concatenate([h["verts"][off[f]:off[f + 1]] for f in s["faces"]])
    assert np.array_equal(np.diff(off)[s["faces"]], s["m"])
    ref = s["verts"]
    err = np.abs(got - ref).max(axis=1) / np.maximum(1.0, np.abs(ref).max(axis=1))
    worst = float(err.max()) if len(err) else 0.0
    assert worst <= vtol, worst
    return worst
