"""am_faces_noalloc (no device allocation, fixed scratch) against am_faces.

Both compute the analytic faces of given cells (Eqn (AnalyticFace) clipped
to the box, vertices by Eqn (VertexEquationSystem)) with the same kernels;
the no-allocation form stages the chain rows in a fixed device array instead
of the context's buffers.  Two calls in a row on one context, the second with
fewer cells, each equal to am_faces bit for bit (the dense chain tile sums
every cell's rows in the same order whatever the batch).
"""
import numpy as np
import pytest

from am_workloads import nets, seeds
from gpu_common import say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def binding():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_10031_amd import binding as B
    return B


def marched_cells(B, net, o, d):
    """Codes and argmax of every cell of a march (faces of the surface)."""
    ctx = B.Context(0).load_net(net)
    ctx.seed_rays(o, d)
    ctx.march(max_cells=1 << 21)
    out = ctx.fetch()
    codes = out["codes"].clone()
    am = out["argmax"].clone()
    torch.cuda.synchronize()
    ctx.close()
    return codes, am


def run_both(B, ctx, codes, am, max_m):
    n = codes.shape[0]
    dev = codes.device
    res = []
    for noalloc in (True, False):
        m = torch.full((n,), -7, dtype=torch.int32, device=dev)
        ids = torch.full((n, max_m), -99, dtype=torch.int32, device=dev)
        verts = torch.full((n, max_m, 3), 7.5, dtype=torch.float64, device=dev)
        flags = torch.full((n,), -1, dtype=torch.int32, device=dev)
        ctx.faces_into(codes, am, None, m, ids, verts, flags, noalloc=noalloc)
        torch.cuda.synchronize()
        res.append((m.cpu().numpy(), ids.cpu().numpy(), verts.cpu().numpy(), flags.cpu().numpy()))
    return res


def assert_same(a, b):
    ma, ia, va, fa = a
    mb, ib, vb, fb = b
    assert np.array_equal(ma, mb)
    assert np.array_equal(fa, fb)
    for f in range(len(ma)):
        k = ma[f]
        assert np.array_equal(ia[f, :k], ib[f, :k]), f
        assert np.array_equal(va[f, :k], vb[f, :k]), f


@pytest.mark.parametrize("name", ["c2", "ensemble"])
def test_faces_noalloc_equals_faces_twice(binding, name):
    B = binding
    if name == "c2":
        net = nets.load_fitted("c2")
        prim = np.load(nets.DATA_DIR + "/c2_primitives.npz")
        o, d = seeds.centre_rays(prim["p0"], 128)
        sizes = (5003, 717)        # several 32 MiB batches with a ragged tail, then fewer cells
    else:
        net = nets.ensemble_net()          # max over 4 heads: argmax is part of each cell
        cs = np.array([c for c, r in nets.ensemble_centres()])
        o, d = seeds.centre_rays(cs, 32)
        sizes = (3001, 257)
    say("faces_noalloc", name)
    codes, am = marched_cells(B, net, o, d)
    assert codes.shape[0] >= sizes[0]
    ctx = B.Context(0).load_net(net)
    rng = np.random.default_rng(5)
    perm = torch.as_tensor(rng.permutation(codes.shape[0]), device=codes.device)
    for k, n in enumerate(sizes):
        sel = perm[k * 1000:k * 1000 + n]
        c = codes[sel].contiguous()
        a = am[sel].contiguous()
        got, ref = run_both(B, ctx, c, a, 32)
        assert (got[0] > 0).sum() > 0.9 * n     # cells of a march have faces
        assert_same(got, ref)
    ctx.close()


def test_faces_noalloc_rejects_bad_arguments(binding):
    B = binding
    net = nets.c1_net()
    ctx = B.Context(0).load_net(net)
    codes = torch.zeros((4, ctx.W), dtype=torch.int64, device="cuda")
    m = torch.empty(4, dtype=torch.int32, device="cuda")
    ids = torch.empty((4, 2), dtype=torch.int32, device="cuda")
    verts = torch.empty((4, 2, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(B.AmError):
        ctx.faces_into(codes, None, None, m, ids, verts, None)   # max_m = 2 is below 3
    ctx.close()
