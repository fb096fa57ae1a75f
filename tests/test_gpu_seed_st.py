"""Sphere-tracing seeds on the GPU (am_seed_points_st) against the oracle.

The seed of a start point is not unique (any surface point of any cell the
path settles in), and near the surface the path crosses many small cells, so
the two sides' different FP64 summation orders may settle in different cells.
A settled point may also lie within rounding of another unit's plane, where
the tie rule decides a bit by summation order.  Bar: every start point
settles or fails on both sides; each GPU seed is a surface point of the
closed cell of its code by the oracle's chain rows for that code (every
oriented constraint <= 1e-12 relative at the point, the head's row = 0 there
within 1e-12); on the exact nets (cube, max-pooled cube: exact dyadic
arithmetic) points and step counts agree; marching from the GPU's seeds gives
the oracle's march from the same seed codes (cells, cycles, adjacency exact;
vertices 1e-9).
"""
import numpy as np
import pytest

from am_workloads import nets
from gpu_common import compare_meshes, fetch_host, say
from oracle import oracle as O

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def binding():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_10031_amd import binding as B
    return B


NETS = {
    "cube": nets.cube_net,
    "maxpool_cube": nets.maxpool_cube_net,
    "c1": nets.c1_net,
    "sphere_like_2x24": lambda: nets.random_sphere_like([24, 24], seed=5, radius=0.6, scale=0.4),
}


@pytest.mark.parametrize("name", list(NETS))
def test_st_seeds_match_oracle(binding, name):
    net = NETS[name]()
    pts = np.random.default_rng(9).uniform(-0.8, 0.8, (48, 3))
    say("st seeds", name)
    ctx = binding.Context(0).load_net(net)
    status, iters, x = ctx.seed_points_st(pts)
    status, iters, x = status.cpu().numpy(), iters.cpu().numpy(), x.cpu().numpy()
    gc, ga, _ = ctx.codes(x)                    # the GPU's code at each settled point
    gc, ga = gc.cpu().numpy().view(np.uint64), ga.cpu().numpy()
    on = O.OracleNet(net)
    seed_codes, seed_am = [], []
    for i, p in enumerate(pts):
        st, xr, code, am, it = on.seed_st(p)
        assert (status[i] == 0) == (st == 0), (i, status[i], st)
        if status[i] != 0:
            continue
        rows = on.chain(gc[i])
        h = np.append(x[i], 1.0)
        scale = np.abs(rows).sum(axis=1) * (1.0 + np.abs(x[i]).max())
        bits = np.array([(int(gc[i][g >> 6]) >> (g & 63)) & 1 for g in range(net.n_hidden)])
        lhs = (1 - 2 * bits) * (rows[:net.n_hidden] @ h)
        assert np.all(lhs <= 1e-12 * scale[:net.n_hidden]), (i, lhs.max())
        assert abs(rows[net.n_hidden + ga[i]] @ h) <= 1e-12 * scale[net.n_hidden + ga[i]]
        if name in ("cube", "maxpool_cube"):
            assert np.max(np.abs(x[i] - xr)) <= 1e-15 and iters[i] == it
        seed_codes.append(gc[i])
        seed_am.append(ga[i])
    assert len(seed_codes) > len(pts) // 2
    st = ctx.march()
    ref = on.march(np.array(seed_codes, np.uint64), np.array(seed_am, np.int32))
    assert st["faces"] == ref.n_faces
    compare_meshes(ref, fetch_host(ctx))
    ctx.close()


def test_st_rejects_bad_inputs(binding):
    ctx = binding.Context(0).load_net(nets.c1_net())
    with pytest.raises(binding.AmError):
        ctx.seed_points_st(np.zeros((1, 3)), max_iter=-1)
    status, _, _ = ctx.seed_points_st(np.zeros((2, 3)), shape_id=np.array([0, 5], np.int32))
    assert status.cpu().numpy().tolist()[1] == 4
    ctx.close()
