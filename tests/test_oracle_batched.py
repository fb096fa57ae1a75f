"""The batched oracle march (the CPU baseline's all-cores leg and the writer
of the golden records) gives the one-cell-at-a-time march's mesh exactly.

Both builds compute every face with the same IEEE operations (the OpenMP
build has contraction off), so the meshes, vertices included, are bit-equal;
the batches only change which thread computes a face.
"""
import numpy as np
import pytest

from am_workloads import nets, seeds
from oracle import oracle as O


def _same(a, b):
    for k in ("codes", "argmax", "offsets", "ids", "nbr"):
        assert np.array_equal(getattr(a, k), getattr(b, k)), k
    assert np.array_equal(a.verts.view(np.uint64), b.verts.view(np.uint64))
    assert a.stats == b.stats


@pytest.mark.parametrize("batch", [1, 7, 4096])
def test_batched_march_equals_sequential_c1(batch):
    net = nets.c1_net()
    on = O.OracleNet(net)
    st, x, code, am = on.seed_ray(np.zeros(3), np.array([1.0, 0.0, 0.0]))
    ref = on.march(code[None], np.array([am]))
    om = O.OracleNet(net, lib_path=O.OMP_LIB_PATH)
    _same(ref, om.march(code[None], np.array([am]), batch=batch))
    _same(ref, on.march(code[None], np.array([am]), batch=batch))


def test_batched_march_equals_sequential_c2_prefix():
    net = nets.load_fitted("c2")
    prim = np.load(nets.DATA_DIR + "/c2_primitives.npz")
    o, d = seeds.centre_rays(prim["p0"], 128)
    on = O.OracleNet(net)
    codes, ams, _, _ = on.seed_rays(o, d)
    ref = on.march(codes, ams, max_cells=12000)
    om = O.OracleNet(net, lib_path=O.OMP_LIB_PATH)
    _same(ref, om.march(codes, ams, max_cells=12000, batch=1000))


def test_faces_batched_equals_face():
    net = nets.c1_net()
    on = O.OracleNet(net)
    om = O.OracleNet(net, lib_path=O.OMP_LIB_PATH)
    st, x, code, am = on.seed_ray(np.zeros(3), np.array([1.0, 0.0, 0.0]))
    mesh = on.march(code[None], np.array([am]), max_cells=500)
    m, ids, verts, flags = om.faces_batched(mesh.codes, mesh.argmax)
    for f in range(mesh.n_faces):
        i, v, _ = mesh.face(f)
        assert m[f] == len(i) and flags[f] == 0
        assert np.array_equal(ids[f, :m[f]], i)
        assert np.array_equal(verts[f, :m[f]].view(np.uint64), v.view(np.uint64))
