"""Mesh invariants used by the tests (Theorem 1 closedness, Euler, area, volume).

Operates on any mesh in the (offsets, ids, verts, nbr) layout: face f owns
entries offsets[f]:offsets[f+1]; entry i is edge i of the face, on constraint
ids[i], starting at vertex verts[i] and bordering face nbr[i] (-1: domain).
"""
import numpy as np


def faces(mesh):
    for f in range(len(mesh.offsets) - 1):
        a, b = mesh.offsets[f], mesh.offsets[f + 1]
        yield f, mesh.ids[a:b], mesh.verts[a:b], mesh.nbr[a:b]


def twin_id(mesh, f, k, n_hidden):
    """Constraint id of the same edge seen from the neighbouring face.

    Hidden-unit edges keep their id; a max-pool comparison edge N+i of a face
    whose argmax is j is the comparison edge N+j of the neighbour (argmax i).
    """
    if n_hidden is None or k < n_hidden:
        return k
    return n_hidden + int(mesh.argmax[f])


def edge_pairing(mesh, atol=1e-9, n_hidden=None):
    """Checks that every non-domain edge is shared by exactly two faces.

    Returns (n_bad, n_domain_edges).  Edge i of face f on constraint k must
    appear in face g = nbr[i] (on the same constraint, or the mirrored
    comparison row for max-pool edges), pointing back to f, with its
    endpoints reversed.
    """
    bad = dom = 0
    off = mesh.offsets
    for f, ids, vs, nb in faces(mesh):
        m = len(ids)
        for i in range(m):
            g = nb[i]
            if g == -1:
                dom += 1
                continue
            if g < 0:
                bad += 1
                continue
            gi = mesh.ids[off[g]:off[g + 1]]
            gv = mesh.verts[off[g]:off[g + 1]]
            gn = mesh.nbr[off[g]:off[g + 1]]
            j = np.nonzero(gi == twin_id(mesh, f, ids[i], n_hidden))[0]
            if len(j) != 1 or gn[j[0]] != f:
                bad += 1
                continue
            j = j[0]
            a0, a1 = vs[i], vs[(i + 1) % m]
            b0, b1 = gv[j], gv[(j + 1) % len(gv)]
            sc = 1.0 + np.abs(a0).max()
            if np.abs(a0 - b1).max() > atol * sc or np.abs(a1 - b0).max() > atol * sc:
                bad += 1
    return bad, dom


def euler(mesh, n_hidden=None):
    """V - E + F with vertices identified through shared edges (combinatorial).

    Corner i of face f is the start of edge i.  Across edge i (to face g,
    matching edge j) the start of edge i equals the end of edge j, i.e.
    corner j+1 of g, and corner i+1 of f equals corner j of g.
    """
    off = mesh.offsets
    n = int(off[-1])
    parent = np.arange(n)

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    def union(a, b):
        a, b = find(a), find(b)
        if a != b:
            parent[a] = b

    n_dom = 0
    for f, ids, vs, nb in faces(mesh):
        m = len(ids)
        for i in range(m):
            g = nb[i]
            if g < 0:
                n_dom += 1
                continue
            gi = mesh.ids[off[g]:off[g + 1]]
            j = int(np.nonzero(gi == twin_id(mesh, f, ids[i], n_hidden))[0][0])
            mg = off[g + 1] - off[g]
            union(off[f] + i, off[g] + (j + 1) % mg)
            union(off[f] + (i + 1) % m, off[g] + j)
    V = len({find(a) for a in range(n)})
    E = (n - n_dom) // 2 + n_dom
    F = len(off) - 1
    return V - E + F, V, E, F


def area_volume(mesh):
    """Total area and the divergence-theorem volume (outward = +grad F)."""
    A = 0.0
    Vol = 0.0
    for f, ids, vs, nb in faces(mesh):
        c = vs.mean(axis=0)
        for i in range(len(vs)):
            cr = np.cross(vs[i] - c, vs[(i + 1) % len(vs)] - c)
            A += 0.5 * np.linalg.norm(cr)
            Vol += np.dot(c, cr) / 6.0
    return A, Vol


def code_key(codes_row, argmax):
    return tuple(int(w) for w in codes_row) + (int(argmax),)


def by_code(mesh):
    """{code key: (ids, verts, neighbour keys)} for mesh comparisons."""
    keys = [code_key(mesh.codes[f], mesh.argmax[f]) for f in range(len(mesh.offsets) - 1)]
    out = {}
    for f, ids, vs, nb in faces(mesh):
        out[keys[f]] = (np.asarray(ids), np.asarray(vs),
                        tuple(keys[g] if g >= 0 else int(g) for g in nb))
    return out
