"""Helpers for the GPU parity tests (device mesh -> host, mesh comparison)."""
import dataclasses
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
