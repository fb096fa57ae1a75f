"""The persistent march (kernel_path 3): one launch in which workgroups take
discovered cells from a device-side queue, compute their chain, clip them and
insert their neighbours into the hash set at once (parallel marching,
Sec. 4.2.2, without steps).

Bars (the oracle records of the single-shape workloads are checked in
test_gpu_golden.py):
* the batched decoder workload: every array of the canonical fetch equals the
  stepped march's (cells, cycles, adjacency exact; vertices bit-equal: the
  chain sums in the same order);
* two persistent marches in a row give the same canonical mesh (the cell ids
  differ from run to run, the mesh does not);
* a cell capacity that is too small ends the march with AM_E_CAPACITY (the
  queue drains, every workgroup leaves), and the context marches again;
* a wait bound set from the host too small for the first round ends the march
  with AM_E_STALL, and the context marches again;
* options the persistent march does not take are refused.
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


KEYS = ("codes", "argmax", "shape", "offsets", "ids", "nbr", "verts")


def test_batched_persistent_equals_stepped(binding):
    sb = nets.c4_batch()
    keep = 24
    o, d, sh = nets.c4_seed_rays(keep)
    say("persistent: c4 batch of", keep, "shapes")
    ctx = binding.Context(0).load_net(sb.net, shape_bias=sb.shape_bias)
    ctx.seed_rays(o, d, shape_id=sh)
    st0 = ctx.march(max_cells=1 << 22)
    ref = ctx.fetch(sorted=True)
    ctx.seed_rays(o, d, shape_id=sh)
    st = ctx.march(max_cells=1 << 22, kernel_path=3)
    got = ctx.fetch(sorted=True)
    assert st["faces"] == st0["faces"] and st["cells"] == st0["cells"]
    for k in KEYS:
        assert torch.equal(got[k], ref[k]), k
    say("persistent c4 faces", st["faces"])
    ctx.close()


def test_persistent_repeats(binding):
    net = nets.load_fitted("c2")
    prim = np.load(nets.DATA_DIR + "/c2_primitives.npz")
    o, d = seeds.centre_rays(prim["p0"], 128)
    ctx = binding.Context(0).load_net(net)
    outs = []
    for r in range(3):
        say("persistent: c2 run", r)
        ctx.seed_rays(o, d)
        st = ctx.march(max_cells=1 << 21, kernel_path=3, time_kernels=(r == 2))
        outs.append((st["faces"], ctx.fetch(sorted=True)))
    for f, out in outs[1:]:
        assert f == outs[0][0]
        for k in KEYS:
            assert torch.equal(out[k], outs[0][1][k]), k
    ctx.close()


def test_persistent_stall_is_reported_and_recovers(binding):
    """A wait bound of four naps, set from the host (wait_limit), makes the
    workgroups that start without a published cell give up before the first
    round has finished anywhere: the march stops with AM_E_STALL, every
    workgroup leaves (each wait stays bounded), and the same context then
    marches with the default bound and gives the whole mesh again.  A
    negative bound is refused before anything runs."""
    net = nets.load_fitted("c2")
    prim = np.load(nets.DATA_DIR + "/c2_primitives.npz")
    o, d = seeds.centre_rays(prim["p0"], 128)
    say("persistent: forced stall on c2")
    ctx = binding.Context(0).load_net(net)
    ctx.seed_rays(o, d)
    ref = ctx.march(max_cells=1 << 21, kernel_path=3)
    ctx.seed_rays(o, d)
    with pytest.raises(binding.AmError) as e:
        ctx.march(max_cells=1 << 21, kernel_path=3, wait_limit=4)
    assert e.value.status == binding.AM_E_STALL
    ctx.seed_rays(o, d)
    st = ctx.march(max_cells=1 << 21, kernel_path=3)
    assert st["faces"] == ref["faces"] and st["cells"] == ref["cells"]
    with pytest.raises(binding.AmError) as e:
        ctx.march(max_cells=1 << 21, kernel_path=3, wait_limit=-1)
    assert e.value.status == binding.AM_E_INVALID
    say("persistent: stall reported, then", st["faces"], "faces")
    ctx.close()


def test_persistent_capacity_overflow(binding):
    net = nets.load_fitted("c2")
    prim = np.load(nets.DATA_DIR + "/c2_primitives.npz")
    o, d = seeds.centre_rays(prim["p0"], 128)
    ctx = binding.Context(0).load_net(net)
    ctx.seed_rays(o, d)
    say("persistent: c2 with room for 20000 cells")
    with pytest.raises(binding.AmError) as e:
        ctx.march(max_cells=20000, kernel_path=3)
    assert "AM_E_CAPACITY" in str(e.value)
    ctx.seed_rays(o, d)
    st = ctx.march(max_cells=1 << 21, kernel_path=3)
    assert st["faces"] == 471884
    ctx.close()


@pytest.mark.parametrize("opts", [dict(precision=1), dict(propose=2), dict(graph_steps=8), dict(max_steps=3),
                                  dict(face_routine=1)])
def test_persistent_refuses_other_forms(binding, opts):
    ctx = binding.Context(0).load_net(nets.c1_net())
    ctx.seed_rays(*seeds.axis_ray())
    with pytest.raises(binding.AmError) as e:
        ctx.march(kernel_path=3, **opts)
    assert "AM_E_INVALID" in str(e.value)
    ctx.close()
