"""The C-ABI boundary: caller allocator, host fetch, asynchronous march,
FP32 network source, head count, ray length.

Each alternative call must give the plain call's mesh exactly: cells,
cycles, adjacency and vertices bit for bit (the same kernels run).
"""
import ctypes as C

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


def c2():
    net = nets.load_fitted("c2")
    prim = np.load(nets.DATA_DIR + "/c2_primitives.npz")
    o, d = seeds.centre_rays(prim["p0"], 128)
    return net, o, d


def host(out):
    from paper_2106_10031_amd.binding import mesh_to_host
    return mesh_to_host(out)


def same_mesh(a, b):
    for k in ("offsets", "ids", "verts", "nbr", "codes", "argmax", "shape"):
        assert np.array_equal(np.asarray(a[k]).view(np.uint8), np.asarray(b[k]).view(np.uint8)), k


def test_allocators_and_host_fetch_agree(binding):
    """Torch's caching allocator and the library's own hipMalloc, device and
    host fetches (discovery and canonical order): identical arrays."""
    B = binding
    net, o, d = c2()
    say("boundary: allocators, host fetch")
    res = {}
    for alloc in ("torch", None):
        ctx = B.Context(0, allocator=alloc).load_net(net)
        ctx.seed_rays(o, d)
        st = ctx.march(max_cells=1 << 21)
        F, V, T, cells = ctx.counts()
        assert (F, V) == (st["faces"], st["face_verts"]) and T == V - 2 * F and cells == st["cells"]
        for sorted_ in (False, True):
            dev = host(ctx.fetch(sorted=sorted_))
            hst = ctx.fetch(sorted=sorted_, where=B.AM_HOST)
            hst["codes"] = hst["codes"].view(np.uint64)
            same_mesh(dev, hst)
            res[(alloc, sorted_)] = hst
        ctx.close()
    same_mesh(res[("torch", True)], res[(None, True)])


def test_async_march_and_wait(binding):
    """opts.async: am_march returns at once, other calls are refused with
    AM_E_STATE while it runs, am_wait returns its stats; the mesh equals a
    blocking march's."""
    B = binding
    net, o, d = c2()
    say("boundary: async march")
    ctx = B.Context(0).load_net(net)
    ctx.seed_rays(o, d)
    ref_st = ctx.march(max_cells=1 << 21)
    ref = host(ctx.fetch(sorted=True))
    ctx.seed_rays(o, d)
    torch.cuda.synchronize()
    assert ctx.march(max_cells=1 << 21, wait=False) is None
    refused = 0
    while ctx.busy():
        try:
            ctx.counts()
        except B.AmError as e:
            assert e.status == B.AM_E_STATE
            refused += 1
            break
    st = ctx.wait()
    assert st["faces"] == ref_st["faces"] and st["steps"] == ref_st["steps"]
    same_mesh(ref, host(ctx.fetch(sorted=True)))
    with pytest.raises(B.AmError):      # nothing left to wait for
        ctx.wait()
    say("async: calls refused while running", refused)
    ctx.close()


def test_f32_source_and_heads(binding):
    """A net handed over as FP32 arrays (exact for the FP32 fit) marches to the
    FP64 hand-over's mesh; a wrong head count is rejected."""
    B = binding
    net, o, d = c2()
    say("boundary: FP32 source")
    got = []
    for dt in (B.AM_F64, B.AM_F32):
        ctx = B.Context(0).load_net(net, dtype=dt)
        ctx.seed_rays(o, d)
        ctx.march(max_cells=1 << 21)
        got.append(host(ctx.fetch(sorted=True)))
        ctx.close()
    same_mesh(got[0], got[1])
    ctx = B.Context(0)
    widths = np.asarray(net.widths, np.int32)
    dst = np.asarray([x for x, _, _ in net.blocks], np.int32)
    src = np.asarray([x for _, x, _ in net.blocks], np.int32)
    ws = [np.ascontiguousarray(W) for _, _, W in net.blocks]
    bs = [np.zeros(3)] + [np.ascontiguousarray(b) for b in net.bias]
    wp = (C.c_void_p * len(ws))(*[w.ctypes.data for w in ws])
    bp = (C.c_void_p * len(bs))(*[b.ctypes.data for b in bs])
    desc = B.NetDesc(len(widths), widths.ctypes.data_as(C.POINTER(C.c_int32)), len(ws),
                     dst.ctypes.data_as(C.POINTER(C.c_int32)), src.ctypes.data_as(C.POINTER(C.c_int32)),
                     wp, bp, 2, B.AM_F64)            # the head layer has 1 unit
    assert ctx.L.am_load_net(ctx.h, C.byref(desc)) == B.AM_E_INVALID
    desc.n_heads, desc.dtype = 1, 7
    assert ctx.L.am_load_net(ctx.h, C.byref(desc)) == B.AM_E_INVALID
    ctx.close()


def test_ray_length(binding):
    """Rays o + t d for t in [0, 2] with half-length directions seed the same
    cells as t in [0, 1] (every bisection point is the same point)."""
    B = binding
    net, o, d = c2()
    say("boundary: t_max")
    ctx = B.Context(0).load_net(net)
    ctx.seed_rays(o, d)
    ctx.march(max_cells=1 << 21)
    a = canonical_codes(host(ctx.fetch(sorted=True)))
    ctx.seed_rays(o, 0.5 * d, t_max=2.0)
    ctx.march(max_cells=1 << 21)
    b = canonical_codes(host(ctx.fetch(sorted=True)))
    assert np.array_equal(a, b)
    ctx.close()


def canonical_codes(h):
    return np.asarray(h["codes"])
