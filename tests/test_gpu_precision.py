"""Precision form: split-BF16 affine chain on matrix cores, FP64 sign tests near
zero (cells whose faces are not certified are redone in FP64) and FP64 vertex
solves.

Bar: cells, cycles and adjacency identical to the FP64 oracle; vertices within
1e-5 relative (|dv|_inf / max(1, |v|_inf)); the split-BF16 rows within 2e-5 of
the FP64 rows (relative to each row's L1 norm).
"""
import os

import numpy as np
import pytest

import meshcheck as MC
from am_workloads import nets, seeds
from gpu_common import compare_meshes, compare_meshes_fast, fetch_host, say
from oracle import oracle as O

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def binding():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_10031_amd import binding as B
    return B


def _fitted(name):
    net = nets.load_fitted(name)
    prim = np.load(os.path.join(nets.DATA_DIR, f"{name}_primitives.npz"))
    o, d = seeds.centre_rays(prim["p0"], 128)
    return net, o, d


@pytest.mark.parametrize("name", ["c1", "c2", "c3"])
def test_split_bf16_rows_close_to_fp64(binding, name):
    net = nets.c1_net() if name == "c1" else _fitted(name)[0]
    on = O.OracleNet(net)
    o, d = seeds.random_rays(16, seed=3) if name == "c1" else _fitted(name)[1:]
    codes, ams, _, _ = on.seed_rays(o[:64], d[:64])
    say("bf16 rows", name, len(codes))
    ctx = binding.Context(0).load_net(net)
    rows = ctx.chain(torch.as_tensor(codes.view(np.int64)).cuda(), precision=1)
    torch.cuda.synchronize()
    rows = rows.cpu().numpy()
    worst = 0.0
    for i, c in enumerate(codes):
        ref = on.chain(c)
        err = np.abs(rows[i] - ref).sum(axis=1) / np.maximum(np.abs(ref).sum(axis=1), 1e-300)
        worst = max(worst, float(err.max()))
    assert worst <= 2e-5, worst


@pytest.mark.parametrize("name", ["c1", "sphere_like_2x24"])
def test_precision_march_small_nets(binding, name):
    net = nets.c1_net() if name == "c1" else nets.random_sphere_like([24, 24], seed=5, radius=0.6, scale=0.4)
    o, d = seeds.random_rays(16, seed=4)
    on = O.OracleNet(net)
    codes, ams, _, _ = on.seed_rays(o, d)
    ref = on.march(codes, ams)
    say("precision march", name, ref.n_faces)
    ctx = binding.Context(0).load_net(net)
    ctx.seed_rays(o, d)
    st = ctx.march(precision=1)
    got = fetch_host(ctx)
    assert st["faces"] == ref.n_faces and st["cells"] == ref.stats["cells"]
    err = compare_meshes(ref, got, vtol=1e-5)
    print(f"{name}: {ref.n_faces} faces, worst vertex error {err:.2e}, escalated {st['escalated']}")


def test_precision_c2_full_equals_oracle(binding):
    net, o, d = _fitted("c2")
    on = O.OracleNet(net)
    codes, ams, _, _ = on.seed_rays(o, d)
    ref = on.march(codes, ams)
    say("precision c2 full", ref.n_faces)
    ctx = binding.Context(0).load_net(net)
    ctx.seed_rays(o, d)
    st = ctx.march(max_cells=1 << 21, precision=1)
    got = fetch_host(ctx)
    assert st["faces"] == ref.n_faces and st["cells"] == ref.stats["cells"]
    err = compare_meshes_fast(ref, got, vtol=1e-5)
    print(f"c2 precision: worst vertex error {err:.2e}, escalated {st['escalated']} of {st['cells']}")


def test_precision_c3_matches_fp64_and_sampled_oracle(binding):
    """8x256 superquadric fit at full size: the two GPU forms agree exactly on
    cells, cycles and adjacency; sampled faces match the oracle one by one."""
    net, o, d = _fitted("c3")
    say("c3 fp64 and precision marches")
    ctx = binding.Context(0).load_net(net)
    ctx.seed_rays(o, d)
    st64 = ctx.march(max_cells=1 << 23, precision=0)
    g64 = fetch_host(ctx)
    ctx.seed_rays(o, d)
    st16 = ctx.march(max_cells=1 << 23, precision=1)
    g16 = fetch_host(ctx)
    assert st64["faces"] == st16["faces"] and st64["degenerate"] == 0
    err = compare_meshes_fast(g64, g16, vtol=1e-5)
    print(f"c3: {st64['faces']} faces, precision form vertex error vs FP64 form {err:.2e}, "
          f"escalated {st16['escalated']} of {st16['cells']}")
    on = O.OracleNet(net)
    rng = np.random.default_rng(11)
    for f in rng.choice(g64.n_faces, 300, replace=False):
        ids, vs, nb = g64.face(f)
        rid, rv, _, fl = on.face(g64.codes[f], g64.argmax[f])
        assert fl == 0 and np.array_equal(ids, rid)
        assert np.max(np.abs(vs - rv)) <= 1e-9 * max(1.0, np.abs(rv).max())
    # closedness (Theorem 1): across every inner edge on unit k, the
    # neighbour's edge on unit k points back (vectorised)
    import gpu_common
    c, a_, mm, ids, vs, nb = gpu_common.canonical(g64)
    face_of = np.repeat(np.arange(len(mm), dtype=np.int64), mm)
    K = np.int64(net.n_hidden + 16)
    keys = face_of * K + ids
    order = np.argsort(keys)
    inner = np.nonzero(nb >= 0)[0]
    want = nb[inner] * K + ids[inner]
    pos = np.searchsorted(keys[order], want)
    assert np.all(pos < len(keys)) and np.array_equal(keys[order][pos], want)
    assert np.array_equal(nb[order][pos], face_of[inner])
