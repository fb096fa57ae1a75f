"""Device-driven marching steps replayed from a captured HIP graph, or
launched one by one with kernel timing.

Bar: the graph march reproduces the oracle's mesh on small nets and batched
shapes (cells, cycles, adjacency exact; vertices 1e-9) and the host-driven
march's mesh on the 6x90 fit exactly; replays reuse the captured graph;
capacity errors surface as AM_E_CAPACITY and a retry with room succeeds.
"""
import numpy as np
import pytest

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


NETS = {
    "c1": nets.c1_net,
    "maxpool_cube": nets.maxpool_cube_net,
    "sphere_like_2x24": lambda: nets.random_sphere_like([24, 24], seed=5, radius=0.6, scale=0.4),
}


@pytest.mark.parametrize("k", [1, 8])
@pytest.mark.parametrize("name", list(NETS))
def test_graph_march_matches_oracle(binding, name, k):
    net = NETS[name]()
    o, d = seeds.random_rays(16, seed=4)
    on = O.OracleNet(net)
    codes, ams, _, _ = on.seed_rays(o, d)
    ref = on.march(codes, ams)
    say("graph march", name, "steps per graph", k)
    ctx = binding.Context(0).load_net(net)
    for _ in range(2):                         # second march replays the same graph
        ctx.seed_rays(o, d)
        st = ctx.march(graph_steps=k)
        assert st["faces"] == ref.n_faces and st["cells"] == ref.stats["cells"]
        compare_meshes(ref, fetch_host(ctx))
    ctx.close()


def test_graph_march_batched(binding):
    sb = nets.latent_sphere_batch([16, 16, 16], reinject=3, latent_dim=8, n_shapes=6, seed=3)
    o, d, sh = [], [], []
    for s in range(sb.n_shapes):
        a, b = seeds.random_rays(12, seed=100 + s)
        o.append(a); d.append(b); sh.append(np.full(12, s, np.int32))
    o, d, sh = np.concatenate(o), np.concatenate(d), np.concatenate(sh)
    say("graph march batched")
    ctx = binding.Context(0).load_net(sb.net, shape_bias=sb.shape_bias)
    ctx.seed_rays(o, d, shape_id=sh)
    ctx.march()
    ref = fetch_host(ctx)
    ctx.seed_rays(o, d, shape_id=sh)
    ctx.march(graph_steps=8)
    compare_meshes_fast(ref, fetch_host(ctx), vtol=0.0)
    ctx.close()


def test_graph_march_c2_equals_host_driven(binding):
    net = nets.load_fitted("c2")
    prim = np.load(nets.DATA_DIR + "/c2_primitives.npz")
    o, d = seeds.centre_rays(prim["p0"], 128)
    say("graph march c2")
    ctx = binding.Context(0).load_net(net)
    ctx.seed_rays(o, d)
    ctx.march(max_cells=1 << 21)
    ref = fetch_host(ctx)
    for k in (4, 16):
        ctx.seed_rays(o, d)
        st = ctx.march(max_cells=1 << 21, graph_steps=k)
        assert st["faces"] == 471884
        compare_meshes_fast(ref, fetch_host(ctx), vtol=0.0)
    ctx.close()


def test_graph_march_capacity_then_retry(binding):
    net = nets.c1_net()
    o, d = seeds.random_rays(16, seed=4)
    ctx = binding.Context(0).load_net(net)
    ctx.seed_rays(o, d)
    with pytest.raises(binding.AmError) as e:
        ctx.march(max_cells=2000, graph_steps=4)
    assert "AM_E_CAPACITY" in str(e.value)
    ctx.seed_rays(o, d)
    st = ctx.march(max_cells=1 << 16, graph_steps=4)
    assert st["faces"] > 2000
    with pytest.raises(binding.AmError):     # pivoting runs host-driven steps only
        ctx.march(graph_steps=4, face_routine=1)
    ctx.close()



def test_graph_march_counts_replays(binding):
    net = nets.c1_net()
    o, d = seeds.random_rays(16, seed=4)
    ctx = binding.Context(0).load_net(net)
    ctx.seed_rays(o, d)
    ref = ctx.march()
    ctx.seed_rays(o, d)
    st = ctx.march(graph_steps=8)
    say("graph replays", st["steps"], st["graph_launches"])
    assert st["faces"] == ref["faces"]
    assert st["graph_launches"] == (st["steps"] + 7) // 8 or st["graph_launches"] == (st["steps"] + 7) // 8 + 1
    ctx.close()


@pytest.mark.parametrize("form", ["fp64", "split"])
@pytest.mark.parametrize("k", [1, 8])
@pytest.mark.parametrize("name", ["c1", "maxpool_cube"])
def test_timed_device_steps_match_oracle(binding, name, k, form):
    """graph_steps with time_kernels: the same device-driven steps launched one
    by one with HIP events; the mesh is the oracle's (vertices 1e-5 for the
    split-BF16 form) and every step that ran is timed once per kernel class."""
    net = NETS[name]()
    o, d = seeds.random_rays(16, seed=4)
    on = O.OracleNet(net)
    codes, ams, _, _ = on.seed_rays(o, d)
    ref = on.march(codes, ams)
    say("timed device steps", name, k, form)
    ctx = binding.Context(0).load_net(net)
    prec = 1 if form == "split" else 0
    for _ in range(2):
        ctx.seed_rays(o, d)
        st = ctx.march(graph_steps=k, time_kernels=True, precision=prec, propose=2 * prec)
        assert st["faces"] == ref.n_faces and st["cells"] == ref.stats["cells"]
        compare_meshes(ref, fetch_host(ctx), vtol=1e-5 if prec else 1e-9)
        assert st["graph_launches"] == 0
        assert st["chain_launches"] == st["steps"] == st["clip_launches"] and st["hash_launches"] == 3 * st["steps"]
        assert st["chain_ms"] > 0.0 and st["clip_ms"] > 0.0 and st["hash_ms"] > 0.0
    ctx.close()


def test_timed_device_steps_c2_equal_host_driven(binding):
    net = nets.load_fitted("c2")
    prim = np.load(nets.DATA_DIR + "/c2_primitives.npz")
    o, d = seeds.centre_rays(prim["p0"], 128)
    say("timed device steps c2")
    ctx = binding.Context(0).load_net(net)
    ctx.seed_rays(o, d)
    host = ctx.march(max_cells=1 << 21, time_kernels=True)
    ref = fetch_host(ctx)
    ctx.seed_rays(o, d)
    st = ctx.march(max_cells=1 << 21, graph_steps=8, time_kernels=True)
    # device-driven steps take at most 16384 cells, so large frontiers take more steps
    assert st["faces"] == 471884 and st["steps"] >= host["steps"]
    assert 0 < st["max_frontier"] and 0 < host["max_frontier"]
    compare_meshes_fast(ref, fetch_host(ctx), vtol=0.0)
    ctx.close()


def test_graph_march_after_reloading_the_net(binding):
    """A context that replayed captured steps for one net and then loads
    another (same or different sizes) must not replay the old graph: its
    nodes hold the freed buffers and the old net by value.  Every march is
    compared with a fresh context's march of the same net."""
    net_a = NETS["c1"]()
    net_b = NETS["sphere_like_2x24"]()
    net_c = nets.random_sphere_like([24, 24], seed=9, radius=0.5, scale=0.4)
    o, d = seeds.random_rays(16, seed=4)
    refs = {}
    for name, net in (("a", net_a), ("b", net_b), ("c", net_c)):
        fresh = binding.Context(0).load_net(net)
        fresh.seed_rays(o, d)
        fresh.march(graph_steps=4)
        refs[name] = fetch_host(fresh)
        fresh.close()
    say("graph march after reload")
    ctx = binding.Context(0)
    for name, net in (("a", net_a), ("b", net_b), ("c", net_c), ("a", net_a)):
        ctx.load_net(net)
        ctx.seed_rays(o, d)
        st = ctx.march(graph_steps=4)
        assert st["faces"] == refs[name].n_faces
        compare_meshes_fast(refs[name], fetch_host(ctx), vtol=0.0)
    ctx.close()
