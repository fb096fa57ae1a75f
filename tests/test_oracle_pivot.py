"""Pins of the oracle's pivoting face routine (Sec. 4.2.1, Alg. 2).

The pivoting routine and the clipping routine compute the same face by
different means (a walk from vertex to vertex with a validity check of each
candidate, against successive halfplane clips of a big square), and neither
calls the other.  Pinned here:
  * brute force: on tiny nets, every face from every one of its edges as the
    start plane equals the face of the naive pair enumeration of Alg. 1;
  * the exact nets (cube; octahedron; the split octahedron, whose extra
    plane x + y = 0 touches four faces only at a vertex; max-pooled cube) and
    a plane section of the box;
  * the clipping routine on generic nets (C1, a max-pooled pair);
  * planted mistakes (no positive-length-edge rule, no orientation fix) fail
    these pins (test_oracle_mutants).
"""
import numpy as np
import pytest

from am_workloads import nets, seeds
from oracle import brute
from oracle import oracle as O
from test_oracle_pins import _maxpool_pair, march_from_ray


def pivot_all_edges(on, code, argmax, ids, vs, verts_tol=0.0):
    """Pivots from every edge of a known face; returns the first mismatch."""
    m = len(ids)
    for i in range(m):
        xs = 0.5 * (vs[i] + vs[(i + 1) % m])
        pid, pv, fl = on.face_pivot(code, argmax, int(ids[i]), xs)
        if fl != 0 or not np.array_equal(pid, ids):
            return (i, ids, pid, fl)
        if np.max(np.abs(pv - vs)) > verts_tol:
            return (i, "verts", float(np.max(np.abs(pv - vs))))
    return None


def check_mesh(on, mesh, limit=None, verts_tol=0.0):
    n = 0
    for f in range(mesh.n_faces):
        ids, vs, _ = mesh.face(f)
        bad = pivot_all_edges(on, mesh.codes[f], mesh.argmax[f], ids, vs, verts_tol)
        assert bad is None, (f, bad)
        n += 1
        if limit and n >= limit:
            break
    return n


def pin_brute(lib_path, net):
    ref = brute.all_faces(net)
    on = O.OracleNet(net, lib_path)
    assert ref
    for (bits, am), (ids, vs) in ref.items():
        code = np.array(brute.bits_to_words(bits, on.W), np.uint64)
        bad = pivot_all_edges(on, code, am, ids, vs, verts_tol=1e-9)
        assert bad is None, (bits, am, bad)


def pin_exact(lib_path, make):
    net = make()
    on = O.OracleNet(net, lib_path)
    _, mesh = march_from_ray(net, lib_path=lib_path)
    assert check_mesh(on, mesh) == mesh.n_faces


BRUTE_NETS = {
    "mlp_5x5": lambda: nets.random_mlp([5, 5], seed=77, bias_std=0.3),
    "shortcut_cube": lambda: nets.shortcut_cube_mlp([4, 4], 301, 0.3),
}


@pytest.mark.parametrize("name", sorted(BRUTE_NETS))
def test_pivot_equals_pair_enumeration(name):
    pin_brute(O.LIB_PATH, BRUTE_NETS[name]())


@pytest.mark.parametrize("make", [nets.cube_net, nets.octahedron_net, nets.octahedron_split_net,
                                  nets.maxpool_cube_net], ids=lambda f: f.__name__)
def test_pivot_on_exact_nets(make):
    pin_exact(O.LIB_PATH, make)


def test_pivot_plane_section_starts_on_a_box_edge():
    net = nets.Net([3, 1], [(1, 0, np.array([[0.0, 0.0, 1.0]]))], [np.array([-0.1])])
    on, mesh = march_from_ray(net, d=(0.0, 0.0, 1.0))
    assert mesh.n_faces == 1 and np.all(mesh.ids < 0)
    assert check_mesh(on, mesh) == 1


@pytest.mark.parametrize("which", ["c1", "maxpool_pair"])
def test_pivot_equals_clip_on_generic_nets(which):
    if which == "c1":
        net = nets.c1_net()
        on, mesh = march_from_ray(net)
        limit = 800
    else:
        net = _maxpool_pair([7, 6], [6], 11)
        on = O.OracleNet(net)
        codes, ams, _, _ = on.seed_rays(*seeds.random_rays(64, seed=9))
        mesh = on.march(codes, ams)
        limit = None
    assert check_mesh(on, mesh, limit) > 0
