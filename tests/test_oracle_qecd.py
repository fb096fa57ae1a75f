"""Pins of the oracle's sequential quadric edge collapse (oracle.qecd;
Sec. 4.4 with Garland and Heckbert's metric).

* The cube net's mesh (26 vertices: face centres and edge midpoints lie on
  one or two of the cube's planes, corners on three) simplifies at zero cost
  to 12 triangles on exactly the 8 corners: area 6, volume 1.
* On a generic closed net the result stays closed and oriented with the same
  Euler characteristic, and its vertices stay near the zero set.
* A planted mistake (collapsing every edge to its midpoint) loses the corners.
"""
import numpy as np
import pytest

from am_workloads import nets, seeds
from oracle import oracle as O
from test_oracle_pins import march_from_ray


def _tris(net, rays=None):
    if rays is None:
        on, mesh = march_from_ray(net)
    else:
        on = O.OracleNet(net)
        codes, ams, _, _ = on.seed_rays(*rays)
        mesh = on.march(codes, ams)
    cv, vx, unp = O.weld(mesh, net.n_hidden)
    assert unp == 0
    return on, vx, O.fan_triangles(mesh.offsets, cv)


def _area_volume(V, T):
    a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    cr = np.cross(b - a, c - a)
    return 0.5 * np.linalg.norm(cr, axis=1).sum(), np.einsum("ij,ij->i", a, cr).sum() / 6.0


def _closed_edges(T, n):
    e = np.concatenate([T[:, [0, 1]], T[:, [1, 2]], T[:, [2, 0]]])
    key = e[:, 0] * n + e[:, 1]
    assert len(np.unique(key)) == len(key)
    assert np.all(np.isin(e[:, 1] * n + e[:, 0], key))
    return len(key) // 2


def test_cube_collapses_to_its_corners():
    _, vx, tri = _tris(nets.cube_net())
    assert len(vx) == 26 and len(tri) == 48
    V, T = O.qecd(vx, tri, 12)
    assert len(V) == 8 and len(T) == 12
    assert np.all(np.abs(np.abs(V) - 0.5) <= 1e-12)
    A, Vol = _area_volume(V, T)
    assert abs(A - 6.0) < 1e-12 and abs(Vol - 1.0) < 1e-12
    _closed_edges(T, len(V))


def test_generic_net_stays_closed_and_near_the_surface():
    net = nets.random_sphere_like([24, 24], seed=5, radius=0.4, scale=0.3)   # closed, inside the box
    on, vx, tri = _tris(net, seeds.random_rays(16, seed=4))
    A0, Vol0 = _area_volume(vx, tri)
    E0 = _closed_edges(tri, len(vx))
    chi0 = len(vx) - E0 + len(tri)
    V, T = O.qecd(vx, tri, len(tri) // 5)
    assert len(T) <= len(tri) // 5 + 2
    E = _closed_edges(T, len(V))
    assert len(V) - E + len(T) == chi0
    A, Vol = _area_volume(V, T)
    assert abs(Vol - Vol0) <= 0.01 * abs(Vol0)
    F = np.array([on.forward(v)[0] for v in V])
    assert np.abs(F).max() <= 0.02


def test_planted_midpoint_mistake_loses_the_corners():
    _, vx, tri = _tris(nets.cube_net())
    V, T = O.qecd(vx, tri, 12, _mutate=1)
    ok = len(V) == 8 and np.all(np.abs(np.abs(V) - 0.5) <= 1e-12)
    assert not ok
