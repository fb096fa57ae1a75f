"""Chain tiles of 4, 8 and 16 cells per workgroup, the gathered tile (K loop
over the units active in any of its four cells), the staged-B tiles (the
producing layer writes the next B operand, masked, into LDS), and the tile
autotuner.

Bar: each variant reproduces the oracle's mesh (cells, cycles, adjacency
exact; vertices 1e-9) on nets with shortcuts, max-pooled heads and per-shape
biases; on the 6x90 fit the dense widths give identical meshes and the
gathered tile the same cells, cycles and adjacency (vertices 1e-9: its sums
run in another order).
"""
import numpy as np
import pytest

from am_workloads import nets, seeds
from gpu_common import canonical, compare_meshes, compare_meshes_fast, fetch_host, say
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
    "c1": nets.c1_net,
    "maxpool_cube": nets.maxpool_cube_net,
    "sphere_like_2x24": lambda: nets.random_sphere_like([24, 24], seed=5, radius=0.6, scale=0.4),
    "shortcut_cube_mlp": lambda: nets.shortcut_cube_mlp([20, 20], seed=2),
}


@pytest.mark.parametrize("groups", [2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("name", list(NETS))
def test_tile_widths_match_oracle(binding, name, groups):
    net = NETS[name]()
    o, d = seeds.random_rays(16, seed=4)
    on = O.OracleNet(net)
    codes, ams, _, _ = on.seed_rays(o, d)
    ref = on.march(codes, ams)
    say("chain tile", name, "groups", groups, ref.n_faces, "faces")
    ctx = binding.Context(0).load_net(net)
    ctx.seed_rays(o, d)
    st = ctx.march(kernel_path=1, chain_groups=groups)
    assert st["faces"] == ref.n_faces
    compare_meshes(ref, fetch_host(ctx))
    ctx.close()


@pytest.mark.parametrize("groups", [2, 3, 4, 5, 6, 7, 8])
def test_tile_widths_batched(binding, groups):
    sb = nets.latent_sphere_batch([16, 16, 16], reinject=3, latent_dim=8, n_shapes=6, seed=3)
    o, d, sh = [], [], []
    for s in range(sb.n_shapes):
        a, b = seeds.random_rays(12, seed=100 + s)
        o.append(a); d.append(b); sh.append(np.full(12, s, np.int32))
    o, d, sh = np.concatenate(o), np.concatenate(d), np.concatenate(sh)
    say("batched chain tile groups", groups)
    ctx = binding.Context(0).load_net(sb.net, shape_bias=sb.shape_bias)
    ctx.seed_rays(o, d, shape_id=sh)
    ctx.march(kernel_path=1, chain_groups=1)
    ref = fetch_host(ctx)
    ctx.seed_rays(o, d, shape_id=sh)
    ctx.march(kernel_path=1, chain_groups=groups)
    compare_meshes_fast(ref, fetch_host(ctx), vtol=0.0 if groups != 5 else 1e-9)
    ctx.close()


def test_tuner_keeps_the_mesh(binding):
    net = nets.load_fitted("c2")
    prim = np.load(nets.DATA_DIR + "/c2_primitives.npz")
    o, d = seeds.centre_rays(prim["p0"], 128)
    say("c2 tiles and tuner")
    ctx = binding.Context(0).load_net(net)
    ctx.seed_rays(o, d)
    ctx.march(max_cells=1 << 21, chain_groups=1)
    ref = fetch_host(ctx)
    for g in (2, 3, 4, 5, 6, 7, 8):
        ctx.seed_rays(o, d)
        ctx.march(max_cells=1 << 21, chain_groups=g)
        compare_meshes_fast(ref, fetch_host(ctx), vtol=0.0 if g != 5 else 1e-9)
    groups, ms = ctx.tune_chain(reps=3)
    say("tuned variants", groups, "ms", np.round(ms, 4).tolist())
    assert all(1 <= g <= binding.CHAIN_VARIANTS for g in groups)
    assert np.all(ms > 0)          # every variant runs on this net
    ctx.seed_rays(o, d)
    ctx.march(max_cells=1 << 21)
    compare_meshes_fast(ref, fetch_host(ctx), vtol=1e-9)
    with pytest.raises(binding.AmError):
        ctx.set_chain_groups([1, binding.CHAIN_VARIANTS + 1, 1, 1])
    ctx.close()


def test_staged_tile_on_wide_layers(binding):
    """Variant 3 stages the previous layer in LDS for widths up to 512: a 2x160
    net (too wide for a ping-pong pair of layers) against the oracle, and
    bit-identical to the dense 4-cell tile (same sums in the same order)."""
    net = nets.random_sphere_like([160, 160], seed=7, radius=0.6, scale=0.4)
    o, d = seeds.random_rays(8, seed=6)
    on = O.OracleNet(net)
    codes, ams, _, _ = on.seed_rays(o, d)
    ref = on.march(codes, ams)
    say("staged tile 2x160", ref.n_faces, "faces")
    ctx = binding.Context(0).load_net(net)
    got = {}
    for g in (1, 3, 6):
        ctx.seed_rays(o, d)
        st = ctx.march(kernel_path=1, chain_groups=g)
        assert st["faces"] == ref.n_faces
        got[g] = fetch_host(ctx)
        compare_meshes_fast(ref, got[g])
    # discovery order differs between marches: compare in canonical face order
    a = canonical(got[1])
    for g in (3, 6):
        b = canonical(got[g])
        assert all(np.array_equal(x, y) for x, y in zip(a, b))
    ctx.close()


@pytest.mark.parametrize("name", ["c2", "c3"])
def test_staged_b_rows_equal_dense_rows(binding, name):
    """am_chain with the staged-B tiles gives the dense 4-cell tile's rows bit
    for bit (same products summed in the same order; FP32-exact weights are
    widened exactly), on cells of the fitted nets, ragged cell counts."""
    net = nets.load_fitted(name)
    prim = np.load(nets.DATA_DIR + f"/{name}_primitives.npz")
    o, d = seeds.centre_rays(prim["p0"], 16)
    ctx = binding.Context(0).load_net(net)
    ctx.seed_rays(o, d)
    ctx.march(max_cells=1 << 22, max_steps=12)
    codes = ctx.fetch()["codes"][:4099].clone()
    say("staged-B rows", name, codes.shape[0], "cells")
    rows = {}
    for g in (1, 6, 7, 8):
        ctx.set_chain_groups([g] * 4)
        rows[g] = ctx.chain(codes).cpu().numpy()
    for g in (6, 7, 8):
        assert np.array_equal(rows[g], rows[1]), g
    ctx.close()
