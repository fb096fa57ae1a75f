"""GPU parity of the welded mesh (am_weld, am_triangles) -- the output
Z = {V, {P}} of Sec. 3 with shared vertices.

Small nets: the GPU's march + weld against the oracle's march + weld.  Faces
are matched by activation code (both sides emit each polygon from the same
starting edge, which the march parity tests check), so corner k of the
canonically ordered GPU mesh is corner k of the oracle's; the vertex
partitions must then be identical (bit-exact), positions within 1e-9, and the
fan triangles identical after relabelling vertices.

Full C2 workload: the partition against the definition (connected components
of the corner identifications, computed on the host from the GPU's own mesh),
every corner within 1e-9 of its vertex, and the edge count from V - E + F.
"""
import ctypes as C

import numpy as np
import pytest

from am_workloads import nets, seeds
from gpu_common import canonical_order, fetch_host, say
from oracle import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def binding():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_10031_amd import binding as B
    return B


def _plane_net():
    return nets.Net([3, 1], [(1, 0, np.array([[0.0, 0.0, 1.0]]))], [np.array([-0.1])])


def _maxpool_pair():
    from test_oracle_pins import _maxpool_pair as mp
    return mp([7, 6], [6], 11)


CASES = {
    "cube": (nets.cube_net, lambda: seeds.random_rays(16, seed=4)),
    "octahedron_split": (nets.octahedron_split_net, lambda: seeds.random_rays(16, seed=4)),
    "maxpool_cube": (nets.maxpool_cube_net, lambda: seeds.random_rays(16, seed=4)),
    "plane": (_plane_net, lambda: (np.zeros((1, 3)), np.array([[0.0, 0.0, 1.0]]))),
    "c1": (nets.c1_net, lambda: seeds.random_rays(16, seed=4)),
    "maxpool_pair": (_maxpool_pair, lambda: seeds.random_rays(64, seed=9)),
}


def _same_partition(a, b):
    pa, pb = {}, {}
    for x, y in zip(a.tolist(), b.tolist()):
        if pa.setdefault(x, y) != y or pb.setdefault(y, x) != x:
            return False
    return True


def _gpu_weld(ctx):
    dev = ctx.fetch()
    cv, vx, unp = ctx.weld(dev)
    tri = ctx.triangles(dev["offsets"], cv)
    torch.cuda.synchronize()
    return dev, cv.cpu().numpy(), vx.cpu().numpy(), unp, tri.cpu().numpy()


@pytest.mark.parametrize("name", list(CASES))
def test_weld_matches_oracle(binding, name):
    make, rays = CASES[name]
    net = make()
    o, d = rays()
    on = O.OracleNet(net)
    codes, ams, _, _ = on.seed_rays(o, d)
    ref = on.march(codes, ams)
    rcv, rvx, runp = O.weld(ref, net.n_hidden)
    rtri = O.fan_triangles(ref.offsets, rcv)
    assert runp == 0
    say("weld", name, ref.n_faces)
    ctx = binding.Context(0).load_net(net)
    ctx.seed_rays(o, d)
    ctx.march()
    got = fetch_host(ctx)
    dev, cv, vx, unp, tri = _gpu_weld(ctx)
    assert unp == 0
    assert len(vx) == len(rvx)
    order, idx = canonical_order(got)
    assert np.array_equal(got.ids[idx], ref.ids), "face cycles differ"
    cvc = cv[idx]
    assert _same_partition(cvc, rcv)
    # ids follow the smallest corner of each class, so they are in first-use order
    first = np.unique(cv, return_index=True)[1]
    assert np.array_equal(np.sort(first), first) and np.array_equal(np.unique(cv), np.arange(len(vx)))
    scale = max(1.0, np.abs(rvx).max()) if len(rvx) else 1.0
    assert np.abs(vx[cvc] - rvx[rcv]).max() <= 1e-9 * scale
    assert np.abs(got.verts - vx[cv]).max() <= 1e-9 * scale
    # triangles: GPU rows of face order[k] relabelled to oracle ids == oracle fan of face k
    g2o = np.empty(len(vx), np.int64)
    g2o[cvc] = rcv
    off = got.offsets
    rows = np.concatenate([np.arange(off[f] - 2 * f, off[f + 1] - 2 * (f + 1)) for f in order]) \
        if len(order) else np.zeros(0, np.int64)
    assert tri.shape == rtri.shape
    assert np.array_equal(g2o[tri[rows]], rtri)


def _definition_partition(mesh, n_hidden):
    """Components of the corner identifications across shared edges (host)."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    off = np.asarray(mesh.offsets, np.int64)
    F = len(off) - 1
    m = np.diff(off)
    n = int(off[-1])
    face = np.repeat(np.arange(F), m)
    local = np.arange(n) - off[face]
    nxt = np.where(local + 1 == m[face], off[face], np.arange(n) + 1)
    ids = mesh.ids.astype(np.int64)
    K = int(ids.max()) + 16
    key = face * K + ids + 8
    srt = np.argsort(key)
    nb = mesh.nbr
    has = nb >= 0
    twin = np.where(ids < n_hidden, ids, n_hidden + mesh.argmax[face].astype(np.int64))
    q = nb[has] * K + twin[has] + 8
    pos = np.searchsorted(key[srt], q)
    assert np.all(key[srt][pos] == q), "an edge has no twin"
    j = srt[pos]
    c = np.nonzero(has)[0]
    a = np.concatenate([c, nxt[c]])
    b = np.concatenate([nxt[j], j])
    g = coo_matrix((np.ones(len(a), np.int8), (a, b)), shape=(n, n))
    _, lab = connected_components(g, directed=False)
    minc = np.full(lab.max() + 1, n, np.int64)
    np.minimum.at(minc, lab, np.arange(n))
    rank = np.empty_like(minc)
    rank[np.argsort(minc)] = np.arange(len(minc))
    return rank[lab]


def test_weld_c2_full_workload(binding):
    net = nets.load_fitted("c2")
    prim = np.load(__import__("os").path.join(nets.DATA_DIR, "c2_primitives.npz"))
    o, d = seeds.centre_rays(prim["p0"], 128)
    say("weld c2 full")
    ctx = binding.Context(0).load_net(net)
    ctx.seed_rays(o, d)
    st = ctx.march(max_cells=1 << 21)
    got = fetch_host(ctx)
    dev, cv, vx, unp, tri = _gpu_weld(ctx)
    assert unp == 0
    ref = _definition_partition(got, net.n_hidden)
    assert np.array_equal(cv, ref)
    assert np.abs(got.verts - vx[cv]).max() <= 1e-9 * max(1.0, np.abs(vx).max())
    F = got.n_faces
    n = len(cv)
    E = (n - st["domain_edges"]) // 2 + st["domain_edges"]
    assert len(tri) == n - 2 * F == st["triangles"]
    # the welded edge set has the same count
    nxt = np.roll(np.arange(n), -1)
    m = np.diff(got.offsets)
    last = got.offsets[1:] - 1
    nxt[last] = got.offsets[:-1]
    u, v = cv, cv[nxt]
    pairs = np.unique(np.minimum(u, v) * len(vx) + np.maximum(u, v))
    assert len(pairs) == E
    say("c2 weld: V", len(vx), "E", E, "F", F, "chi", len(vx) - E + F)


def test_weld_edge_cases_and_scratch_reuse(binding):
    net = nets.c1_net()
    ctx = binding.Context(0).load_net(net)
    say("weld edge cases")
    # empty mesh
    e = dict(offsets=torch.zeros(1, dtype=torch.int64, device="cuda"),
             ids=torch.zeros(0, dtype=torch.int32, device="cuda"),
             nbr=torch.zeros(0, dtype=torch.int64, device="cuda"),
             verts=torch.zeros((0, 3), dtype=torch.float64, device="cuda"),
             argmax=torch.zeros(0, dtype=torch.int32, device="cuda"))
    cv, vx, unp = ctx.weld(e)
    assert cv.shape[0] == 0 and vx.shape[0] == 0 and unp == 0
    assert ctx.triangles(e["offsets"], cv).shape[0] == 0
    # a big mesh, then a small one on the same context (scratch is reused)
    o, d = seeds.random_rays(16, seed=4)
    ctx.seed_rays(o, d)
    ctx.march()
    _, cv1, vx1, _, _ = _gpu_weld(ctx)
    ctx.load_net(nets.cube_net())
    ctx.seed_rays(o, d)
    ctx.march()
    _, cv2, vx2, unp2, _ = _gpu_weld(ctx)
    assert len(vx2) == 26 and unp2 == 0 and len(vx1) > 1000
    # too few vxyz rows: an error, but corner ids and the count are still given
    dev = ctx.fetch()
    F = dev["offsets"].shape[0] - 1
    n = dev["ids"].shape[0]
    cvt = torch.empty(n, dtype=torch.int64, device="cuda")
    vxt = torch.empty((4, 3), dtype=torch.float64, device="cuda")
    nv, up = C.c_int64(), C.c_int64()
    P = lambda t: C.c_void_p(t.data_ptr())
    L = ctx.L
    rc = L.am_weld(ctx.h, F, P(dev["offsets"]), P(dev["ids"]), P(dev["nbr"]), P(dev["argmax"]), P(dev["verts"]),
                   n, P(cvt), P(vxt), 4, C.byref(nv), C.byref(up))
    assert rc != 0 and nv.value == 26
    assert np.array_equal(cvt.cpu().numpy(), cv2)
    # offsets that do not end at the corner count are rejected before any launch
    rc = L.am_weld(ctx.h, F, P(dev["offsets"]), P(dev["ids"]), P(dev["nbr"]), P(dev["argmax"]), P(dev["verts"]),
                   n - 1, P(cvt), None, 0, C.byref(nv), C.byref(up))
    assert rc != 0
