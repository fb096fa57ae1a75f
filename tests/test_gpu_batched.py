"""Batched form: many shapes sharing weights, marched together in one frontier.

Bar: every shape's part of the batched march equals (a) the oracle's march of
that shape's own network and (b) the GPU's single-shape march of it (cell
set, cycles, adjacency exact; vertices 1e-9).
"""
import numpy as np
import pytest

import meshcheck as MC
from am_workloads import nets, seeds
from gpu_common import HostMesh, compare_meshes, fetch_host, say
from oracle import oracle as O

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def binding():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_10031_amd import binding as B
    return B


def _split_by_shape(ctx):
    from paper_2106_10031_amd.binding import mesh_to_host
    h = mesh_to_host(ctx.fetch())
    out = {}
    shapes = h["shape"]
    off = h["offsets"]
    for s in np.unique(shapes):
        fs = np.nonzero(shapes == s)[0]
        remap = {int(f): i for i, f in enumerate(fs)}
        offs, ids, verts, nbr = [0], [], [], []
        for f in fs:
            a, b = off[f], off[f + 1]
            ids.append(h["ids"][a:b])
            verts.append(h["verts"][a:b])
            nbr.append([remap[int(g)] if g >= 0 else int(g) for g in h["nbr"][a:b]])
            offs.append(offs[-1] + (b - a))
        out[int(s)] = HostMesh(h["codes"][fs], h["argmax"][fs], np.asarray(offs), np.concatenate(ids),
                               np.concatenate(verts), np.concatenate(nbr).astype(np.int64))
    return out


def _rays(S, per):
    o, d, sh = [], [], []
    for s in range(S):
        a, b = seeds.random_rays(per, seed=100 + s)
        o.append(a); d.append(b); sh.append(np.full(per, s, np.int32))
    return np.concatenate(o), np.concatenate(d), np.concatenate(sh)


@pytest.mark.parametrize("path", [1, 2], ids=["split", "fused"])
def test_batched_equals_oracle_and_single_shape(binding, path):
    sb = nets.latent_sphere_batch([16, 16, 16], reinject=3, latent_dim=8, n_shapes=6, seed=3)
    o, d, sh = _rays(sb.n_shapes, 12)
    say("batched march", sb.n_shapes, "shapes, path", path)
    ctx = binding.Context(0).load_net(sb.net, shape_bias=sb.shape_bias)
    assert ctx.S == sb.n_shapes
    ctx.seed_rays(o, d, shape_id=sh)
    st = ctx.march(kernel_path=path)
    got = _split_by_shape(ctx)
    total = 0
    for s in range(sb.n_shapes):
        net = sb.shape_net(s)
        on = O.OracleNet(net)
        m = sh == s
        codes, ams, _, _ = on.seed_rays(o[m], d[m])
        ref = on.march(codes, ams)
        compare_meshes(ref, got[s])
        total += ref.n_faces
        single = binding.Context(0).load_net(net)
        single.seed_rays(o[m], d[m])
        single.march(kernel_path=path)
        compare_meshes(ref, fetch_host(single))
        bad, _ = MC.edge_pairing(got[s], n_hidden=net.n_hidden)
        assert bad == 0
    assert st["faces"] == total


def test_shape_ids_are_validated(binding):
    sb = nets.latent_sphere_batch([8, 8], reinject=2, latent_dim=4, n_shapes=3, seed=5)
    say("shape id validation")
    ctx = binding.Context(0).load_net(sb.net, shape_bias=sb.shape_bias)
    o, d = seeds.random_rays(4, seed=1)
    status = ctx.seed_rays(o, d, shape_id=np.array([0, 1, 7, -1], np.int32))
    torch.cuda.synchronize()
    st = status.cpu().numpy()
    assert st[2] == 3 and st[3] == 3
    codes, am, F = ctx.codes(o, shape_id=np.array([0, 2, 3, 1], np.int32))
    torch.cuda.synchronize()
    assert am.cpu().numpy()[2] == -1 and np.isnan(F.cpu().numpy()[2])


def test_wide_decoder_batch_equals_single_shape_marches(binding):
    """The 64-shape decoder's first 12 shapes (the smallest boxes): each shape's part
    of one batched march equals that shape's own GPU march (cells, cycles,
    adjacency exact; vertices bit-equal: same rows, same solves)."""
    from gpu_common import compare_meshes_fast
    sb = nets.c4_batch()
    keep = 12
    o, d, sh = nets.c4_seed_rays(keep)
    say("c4 batch of", keep, "shapes")
    ctx = binding.Context(0).load_net(sb.net, shape_bias=sb.shape_bias)
    ctx.seed_rays(o, d, shape_id=sh)
    st = ctx.march(max_cells=1 << 20)
    got = _split_by_shape(ctx)
    total = 0
    for s in range(keep):
        m = sh == s
        ctx.seed_rays(o[m], d[m], shape_id=sh[m])
        ctx.march(max_cells=1 << 20)
        one = fetch_host(ctx)
        compare_meshes_fast(one, got[s], vtol=0.0)
        total += one.n_faces
    assert st["faces"] == total
    ctx.close()


@pytest.mark.parametrize("graph", [0, 8], ids=["host", "graph"])
@pytest.mark.parametrize("propose", [2, 1], ids=["distance", "scorer"])
def test_wide_decoder_batch_bf16_with_proposals_equals_plain(binding, propose, graph):
    """All three growth patterns at once on the decoder batch's first 12
    shapes: one batched march with the split-BF16 chain and proposed clip
    lines (ordered by distance, or by an untrained scorer: proposals are
    always checked, so any scorer gives the exact face set) against the
    plain FP64 batched march.  Cells, cycles and adjacency exact; vertices
    within the precision form's 1e-5, at the default certificate (its row
    error measured for this decoder on the march's seed cells); host-driven
    steps and device-driven steps replayed from a captured graph."""
    from gpu_common import compare_meshes_fast
    from paper_2106_10031_amd.learn import init_params
    sb = nets.c4_batch()
    keep = 12
    o, d, sh = nets.c4_seed_rays(keep)
    say("c4 batch of", keep, "shapes, bf16 + proposals", propose)
    ctx = binding.Context(0).load_net(sb.net, shape_bias=sb.shape_bias)
    ctx.seed_rays(o, d, shape_id=sh)
    st0 = ctx.march(max_cells=1 << 20)
    ref = fetch_host(ctx)
    if propose == 1:
        ctx.prop_set(init_params(7).astype(np.float32), k=16, rho=6.0)
    ctx.seed_rays(o, d, shape_id=sh)
    st = ctx.march(max_cells=1 << 20, precision=1, propose=propose, graph_steps=graph)
    got = fetch_host(ctx)
    assert st["faces"] == st0["faces"]
    compare_meshes_fast(ref, got, vtol=1e-5)
    assert st["prop_cells"] > 0
    say("escalated", st["escalated"], "proposed", st["prop_cells"], "accepted", st["prop_accepted"])
    ctx.close()
