"""Pins of the oracle's welded mesh (oracle.weld, oracle.fan_triangles).

The welded form is the output Z = {V, {P}} of Sec. 3: one vertex array and
polygons that index it.  Pinned against what does not come from the weld:
  * closed forms of hand-built nets: the vertex set of the cube net is
    {-1/2, 0, 1/2}^3 without the centre, the octahedron's is +-0.75 e_i, the
    max-pooled cube's the 8 corners; edge counts from the welded polygons and
    V - E + F = 2; triangle-fan area and enclosed volume against the closed
    forms (the signed volume also pins the triangles' winding);
  * an open surface (a plane through the box): 4 corners of the box section;
  * brute force on generic nets: corners at the same point (within 1e-9) are
    exactly the corners of one vertex;
  * a planted mistake in the corner pairing fails the closed forms.
"""
import math

import numpy as np
import pytest
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components
from scipy.spatial import cKDTree

from am_workloads import nets, seeds
from oracle import oracle as O
from test_oracle_pins import _maxpool_pair, march_from_ray


def _grid_points(vals, drop_origin=False):
    pts = np.array([(a, b, c) for a in vals for b in vals for c in vals], float)
    if drop_origin:
        pts = pts[np.abs(pts).sum(axis=1) > 0]
    return pts


def _same_point_set(a, b, tol=1e-12):
    a = np.asarray(a)
    b = np.asarray(b)
    if a.shape != b.shape:
        return False
    d = np.abs(a[:, None, :] - b[None, :, :]).max(axis=2)
    return bool((d.min(axis=1) <= tol).all() and (d.min(axis=0) <= tol).all())


def _edges(off, cv):
    """Distinct undirected vertex pairs over all polygon edges."""
    e = set()
    for f in range(len(off) - 1):
        a0, m = int(off[f]), int(off[f + 1] - off[f])
        for i in range(m):
            u, v = int(cv[a0 + i]), int(cv[a0 + (i + 1) % m])
            e.add((min(u, v), max(u, v)))
    return e


def _octa(r):
    return np.array([s * r * np.eye(3)[k] for k in range(3) for s in (1, -1)])


EXACT = {
    "cube": (nets.cube_net, 56, 6.0, 1.0, lambda: _grid_points([-0.5, 0.0, 0.5], drop_origin=True)),
    "octahedron": (nets.octahedron_net, 12, 4.0 * math.sqrt(3.0) * 0.75 ** 2, (4.0 / 3.0) * 0.75 ** 3,
                   lambda: _octa(0.75)),
    "octahedron_split": (nets.octahedron_split_net, 18, 4.0 * math.sqrt(3.0) * 0.75 ** 2,
                         (4.0 / 3.0) * 0.75 ** 3,
                         lambda: np.vstack([_octa(0.75), [[0.375, -0.375, 0.0], [-0.375, 0.375, 0.0]]])),
    "maxpool_cube": (nets.maxpool_cube_net, 12, 6.0, 1.0, lambda: _grid_points([-0.5, 0.5])),
}


@pytest.mark.parametrize("name", sorted(EXACT))
def test_exact_nets_vertex_sets(name):
    make, E, area, vol, pts = EXACT[name]
    net = make()
    _, mesh = march_from_ray(net)
    cv, vx, unp = O.weld(mesh, net.n_hidden)
    assert unp == 0
    assert _same_point_set(vx, pts()), name
    # every corner sits at its vertex
    assert np.abs(mesh.verts - vx[cv]).max() <= 1e-15
    e = _edges(mesh.offsets, cv)
    assert len(e) == E
    assert len(vx) - len(e) + mesh.n_faces == 2
    tri = O.fan_triangles(mesh.offsets, cv)
    assert len(tri) == int(np.sum(np.diff(mesh.offsets) - 2))
    a, b, c = vx[tri[:, 0]], vx[tri[:, 1]], vx[tri[:, 2]]
    cr = np.cross(b - a, c - a)
    assert abs(0.5 * np.linalg.norm(cr, axis=1).sum() - area) < 1e-12
    # divergence theorem with the outward (+grad F) winding of the faces
    assert abs(np.einsum("ij,ij->i", a, cr).sum() / 6.0 - vol) < 1e-12


def test_open_surface_plane_section():
    net = nets.Net([3, 1], [(1, 0, np.array([[0.0, 0.0, 1.0]]))], [np.array([-0.1])])
    _, mesh = march_from_ray(net, d=(0.0, 0.0, 1.0))
    cv, vx, unp = O.weld(mesh, net.n_hidden)
    assert unp == 0 and mesh.n_faces == 1
    assert _same_point_set(vx, [(sx, sy, 0.1) for sx in (-1.0, 1.0) for sy in (-1.0, 1.0)])
    assert len(O.fan_triangles(mesh.offsets, cv)) == 2


def _geometric_partition(verts, tol=1e-9):
    pairs = cKDTree(verts).query_pairs(tol, output_type="ndarray")
    n = len(verts)
    g = coo_matrix((np.ones(len(pairs)), (pairs[:, 0], pairs[:, 1])), shape=(n, n)) if len(pairs) else \
        coo_matrix((n, n))
    _, lab = connected_components(g, directed=False)
    return lab


def _same_partition(a, b):
    """Two labelings induce the same partition iff label pairs are a bijection."""
    pa = {}
    pb = {}
    for x, y in zip(a.tolist(), b.tolist()):
        if pa.setdefault(x, y) != y or pb.setdefault(y, x) != x:
            return False
    return True


@pytest.mark.parametrize("which", ["c1", "maxpool"])
def test_weld_equals_geometric_clustering_on_generic_nets(which):
    if which == "c1":
        net = nets.c1_net()
        on, mesh = march_from_ray(net)
    else:
        net = _maxpool_pair([7, 6], [6], 11)
        on = O.OracleNet(net)
        o, d = seeds.random_rays(64, seed=9)
        codes, ams, pts, sts = on.seed_rays(o, d)
        mesh = on.march(codes, ams)
    cv, vx, unp = O.weld(mesh, net.n_hidden)
    assert unp == 0
    geo = _geometric_partition(mesh.verts)
    assert _same_partition(cv, geo)
    assert np.abs(mesh.verts - vx[cv]).max() <= 1e-9


def test_planted_pairing_mistake_fails_the_closed_form():
    net = nets.cube_net()
    _, mesh = march_from_ray(net)
    cv, vx, _ = O.weld(mesh, net.n_hidden, _mutate=1)
    assert not _same_point_set(vx, EXACT["cube"][4]())
    assert np.abs(mesh.verts - vx[cv]).max() > 0.1
