"""GPU parity of the pivoting face routine (Sec. 4.2.1; am_march_opts.face_routine = 1).

The march with faces traced vertex by vertex from their entry edges must give
the oracle's mesh: cell set, cycles and adjacency bit-exact, vertices within
1e-9 relative, on the exact nets (degenerate vertices where four planes
meet, a plane that touches faces only at a vertex), generic nets, a max-pool
union, and the full C2 workload.  The oracle's own pivoting routine is pinned
to its clipping routine in the CPU tests, so the face has one definition.
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


def _maxpool_pair():
    from test_oracle_pins import _maxpool_pair as mp
    return mp([7, 6], [6], 11)


NETS = {
    "cube": nets.cube_net,
    "octahedron_split": nets.octahedron_split_net,
    "maxpool_cube": nets.maxpool_cube_net,
    "c1": nets.c1_net,
    "sphere_like_2x24": lambda: nets.random_sphere_like([24, 24], seed=5, radius=0.6, scale=0.4),
    "maxpool_pair": _maxpool_pair,
}


@pytest.mark.parametrize("name", list(NETS))
def test_pivot_march_matches_oracle(binding, name):
    net = NETS[name]()
    o, d = seeds.random_rays(16 if name != "maxpool_pair" else 64, seed=4)
    on = O.OracleNet(net)
    codes, ams, _, _ = on.seed_rays(o, d)
    ref = on.march(codes, ams)
    say("pivot march", name, ref.n_faces)
    ctx = binding.Context(0).load_net(net)
    ctx.seed_rays(o, d)
    st = ctx.march(face_routine=1)
    got = fetch_host(ctx)
    assert st["faces"] == ref.n_faces and st["cells"] == ref.stats["cells"]
    compare_meshes(ref, got)
    bad, _ = MC.edge_pairing(got, n_hidden=net.n_hidden)
    assert bad == 0
    assert st["pivot_cells"] + st["pivot_fallback"] == st["cells"]
    entered = st["cells"] - st["seed_cells"]
    if name in ("c1", "sphere_like_2x24"):
        assert st["pivot_cells"] >= 0.9 * entered, st
    elif entered > 0 and name != "maxpool_cube":
        assert st["pivot_cells"] > 0, st


def test_pivot_c2_full_workload_equals_oracle(binding):
    net = nets.load_fitted("c2")
    prim = np.load(os.path.join(nets.DATA_DIR, "c2_primitives.npz"))
    o, d = seeds.centre_rays(prim["p0"], 128)
    on = O.OracleNet(net)
    codes, ams, _, _ = on.seed_rays(o, d)
    ref = on.march(codes, ams)
    say("pivot c2 full vs oracle", ref.n_faces)
    ctx = binding.Context(0).load_net(net)
    ctx.seed_rays(o, d)
    st = ctx.march(max_cells=1 << 21, face_routine=1)
    got = fetch_host(ctx)
    assert st["faces"] == ref.n_faces and st["cells"] == ref.stats["cells"]
    compare_meshes_fast(ref, got)
    say("pivot c2: walked", st["pivot_cells"], "clipped", st["pivot_fallback"])
    assert st["pivot_cells"] > 0.99 * st["cells"]


def test_pivot_rejects_other_forms(binding):
    net = nets.c1_net()
    ctx = binding.Context(0).load_net(net)
    o, d = seeds.random_rays(4, seed=1)
    ctx.seed_rays(o, d)
    for kw in (dict(precision=1), dict(propose=2), dict(graph_steps=4), dict(kernel_path=2)):
        with pytest.raises(binding.AmError):
            ctx.march(face_routine=1, **kw)
    with pytest.raises(binding.AmError):
        ctx.march(face_routine=2)
