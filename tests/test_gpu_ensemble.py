"""A max-pooled ensemble of 4 depth-4 sub-networks (Sec. 5.2; the local
decoders of Table 7), marched on the union of the sub-networks' insides.

Bar: the GPU's mesh equals the oracle's (cells incl. argmax, cycles,
adjacency exact; vertices 1e-9) with the dense and the gathered chain tile;
every edge pairs up (comparison edges included).
"""
import numpy as np
import pytest

import meshcheck as MC
from am_workloads import nets, seeds
from gpu_common import compare_meshes_fast, fetch_host, say
from oracle import oracle as O

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def binding():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_10031_amd import binding as B
    return B


@pytest.fixture(scope="module")
def case():
    net = nets.ensemble_net(width=16)
    cs = np.array([c for c, r in nets.ensemble_centres()])
    o, d = seeds.centre_rays(cs, 32)
    on = O.OracleNet(net)
    codes, ams, _, _ = on.seed_rays(o, d)
    return net, o, d, on.march(codes, ams)


@pytest.mark.parametrize("variant", [1, 5])
def test_ensemble_matches_oracle(binding, case, variant):
    net, o, d, ref = case
    say("ensemble 4 x D4-W16, chain variant", variant, ref.n_faces, "faces")
    ctx = binding.Context(0).load_net(net)
    ctx.seed_rays(o, d)
    st = ctx.march(max_cells=1 << 20, chain_groups=variant)
    got = fetch_host(ctx)
    assert st["faces"] == ref.n_faces
    compare_meshes_fast(ref, got, vtol=1e-9)
    assert len(np.unique(got.argmax)) == net.n_heads
    bad, _ = MC.edge_pairing(got, n_hidden=net.n_hidden)
    assert bad == 0
    ctx.close()
