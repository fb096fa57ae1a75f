"""Quadric edge-collapse simplification (am_simplify; Sec. 4.4) of the
welded triangle mesh of a march.

The result depends on collapse order, so it is checked against what does not:
  * the cube net's mesh (48 triangles, 26 vertices: face centres and edge
    midpoints lie on one or two planes, corners on three) simplifies at zero
    cost to 12 triangles on the 8 corners, with area 6 and volume 1 exactly;
  * against the CPU reference's sequential collapse on a closed net: the
    same counts and topology, vertex error and volume on a par;
  * edge cases: bad input triangles, targets out of reach either way, frozen
    vertices, and the argument checks;
  * on C1 and C2 at 10 %: the triangle count reaches the target, the mesh
    stays closed and consistently oriented (each undirected edge in exactly
    two triangles, once each way), the Euler characteristic is unchanged,
    every vertex stays near the zero set (|F| from the CPU reference's
    forward pass) and the enclosed volume changes by under 1 %.
"""
import os

import numpy as np
import pytest

from am_workloads import nets, seeds
from gpu_common import say
from oracle import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def binding():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_10031_amd import binding as B
    return B


def _welded_tris(ctx):
    dev = ctx.fetch()
    cv, vx, unp = ctx.weld(dev)
    assert unp == 0
    tri = ctx.triangles(dev["offsets"], cv)
    return vx.contiguous(), tri.contiguous()


def _area_volume(V, T):
    a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    cr = np.cross(b - a, c - a)
    return 0.5 * np.linalg.norm(cr, axis=1).sum(), np.einsum("ij,ij->i", a, cr).sum() / 6.0


def _check_closed(T, n_verts):
    e = np.concatenate([T[:, [0, 1]], T[:, [1, 2]], T[:, [2, 0]]])
    key = e[:, 0] * n_verts + e[:, 1]
    assert len(np.unique(key)) == len(key), "a directed edge appears twice"
    rev = e[:, 1] * n_verts + e[:, 0]
    assert np.all(np.isin(rev, key)), "an edge has no opposite half"
    return len(key) // 2


def test_cube_simplifies_to_its_corners(binding):
    net = nets.cube_net()
    ctx = binding.Context(0).load_net(net)
    o, d = seeds.random_rays(16, seed=4)
    ctx.seed_rays(o, d)
    ctx.march()
    vx, tri = _welded_tris(ctx)
    say("simplify cube", vx.shape[0], tri.shape[0])
    v2, t2, rounds, bad = ctx.simplify(vx, tri, 12)
    V = v2.cpu().numpy()
    T = t2.cpu().numpy()
    assert bad == 0 and len(T) == 12 and len(V) == 8, (len(T), len(V), rounds)
    assert np.all(np.abs(np.abs(V) - 0.5) <= 1e-12)
    A, Vol = _area_volume(V, T)
    assert abs(A - 6.0) < 1e-12 and abs(Vol - 1.0) < 1e-12
    _check_closed(T, len(V))


def _case(name):
    if name == "c1":
        return nets.c1_net(), seeds.random_rays(16, seed=4), 2
    net = nets.load_fitted("c2")
    prim = np.load(os.path.join(nets.DATA_DIR, "c2_primitives.npz"))
    return net, seeds.centre_rays(prim["p0"], 128), 4


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_simplify_to_ten_percent(binding, name):
    net, (o, d), chi = _case(name)
    ctx = binding.Context(0).load_net(net)
    ctx.seed_rays(o, d)
    ctx.march(max_cells=1 << 21)
    vx, tri = _welded_tris(ctx)
    T0 = tri.shape[0]
    V0 = vx.cpu().numpy()
    A0, Vol0 = _area_volume(V0, tri.cpu().numpy())
    target = T0 // 10
    say("simplify", name, T0, "->", target)
    v2, t2, rounds, bad = ctx.simplify(vx, tri, target)
    V = v2.cpu().numpy()
    T = t2.cpu().numpy()
    say("simplified", name, len(T), "triangles", len(V), "vertices", rounds, "rounds")
    assert bad == 0
    assert len(T) <= target + 2
    E = _check_closed(T, len(V))
    assert len(V) - E + len(T) == chi
    A, Vol = _area_volume(V, T)
    assert abs(Vol - Vol0) <= 0.01 * abs(Vol0)
    on = O.OracleNet(net)
    pick = np.random.default_rng(0).choice(len(V), size=min(2000, len(V)), replace=False)
    F = np.array([on.forward(V[i])[0] for i in pick])
    say("max |F| at simplified vertices", float(np.abs(F).max()))
    assert np.abs(F).max() <= 0.02


def test_simplify_matches_the_sequential_reference(binding):
    """Parallel rounds against the oracle's sequential collapse (cheapest
    edge first) on the same closed net at 20 %: the same triangle count, and
    vertex error, volume and topology on a par (the two orders differ, so
    the meshes do)."""
    net = nets.random_sphere_like([24, 24], seed=5, radius=0.4, scale=0.3)
    rays = seeds.random_rays(16, seed=4)
    on = O.OracleNet(net)
    codes, ams, _, _ = on.seed_rays(*rays)
    mesh = on.march(codes, ams)
    cv, rvx, _ = O.weld(mesh, net.n_hidden)
    rtri = O.fan_triangles(mesh.offsets, cv)
    target = len(rtri) // 5
    RV, RT = O.qecd(rvx, rtri, target)
    say("simplify vs reference", len(rtri), "->", target)
    ctx = binding.Context(0).load_net(net)
    ctx.seed_rays(*rays)
    ctx.march()
    vx, tri = _welded_tris(ctx)
    assert tri.shape[0] == len(rtri)
    v2, t2, rounds, bad = ctx.simplify(vx, tri, target)
    V = v2.cpu().numpy()
    T = t2.cpu().numpy()
    assert len(T) == len(RT) and len(V) == len(RV)
    E, RE = _check_closed(T, len(V)), _check_closed(RT, len(RV))
    assert len(V) - E + len(T) == len(RV) - RE + len(RT)
    _, vol = _area_volume(V, T)
    _, rvol = _area_volume(RV, RT)
    assert abs(vol - rvol) <= 0.005 * abs(rvol)
    F = np.abs([on.forward(v)[0] for v in V]).max()
    RF = np.abs([on.forward(v)[0] for v in RV]).max()
    say("max |F|: GPU", F, "reference", RF)
    assert F <= 2.0 * RF + 1e-6


def test_simplify_edge_cases(binding):
    """Bad input triangles are dropped and counted; a target at or above the
    live count leaves the mesh as it is; a target nothing can reach stops
    when no edge can collapse, with the mesh still closed; sizes beyond the
    32-bit ids and other bad arguments are rejected before any launch."""
    import ctypes as C
    net = nets.cube_net()
    ctx = binding.Context(0).load_net(net)
    o, d = seeds.random_rays(16, seed=4)
    ctx.seed_rays(o, d)
    ctx.march()
    vx, tri = _welded_tris(ctx)
    nV, nT = vx.shape[0], tri.shape[0]
    say("simplify edge cases", nV, nT)
    junk = torch.tensor([[0, 0, 1], [0, 1, nV], [-1, 2, 3]], dtype=torch.int64, device="cuda")
    tri_bad = torch.cat([tri, junk]).contiguous()
    for target in (nT, 10 * nT):
        v2, t2, rounds, bad = ctx.simplify(vx, tri_bad, target)
        assert bad == 3 and rounds == 0
        assert torch.equal(t2, tri) and torch.equal(v2, vx)
    v2, t2, rounds, bad = ctx.simplify(vx, tri, 0)
    V, T = v2.cpu().numpy(), t2.cpu().numpy()
    assert bad == 0 and rounds >= 1 and 2 <= len(T) <= 12
    E = _check_closed(T, len(V))
    assert len(V) - E + len(T) == 2
    # a boundary flag on every vertex freezes the mesh
    frozen = torch.ones(nV, dtype=torch.uint8, device="cuda")
    v2, t2, rounds, bad = ctx.simplify(vx, tri, 12, boundary=frozen)
    assert torch.equal(t2, tri) and rounds == 1
    # argument checks (no launch: the sizes are refused first)
    P = lambda t: C.c_void_p(t.data_ptr())
    vo = torch.empty_like(vx)
    to = torch.empty_like(tri)
    nv, nt, r, nb = C.c_int64(), C.c_int64(), C.c_int32(), C.c_int64()
    L = ctx.L

    def call(V, T, target, max_rounds):
        return L.am_simplify(ctx.h, V, P(vx), T, P(tri), None, target, max_rounds, P(vo), P(to), C.byref(nv),
                             C.byref(nt), C.byref(r), C.byref(nb))

    assert call(1 << 30, nT, 12, 0) != 0
    assert call(nV, 1 << 30, 12, 0) != 0
    assert call(nV, 0, 12, 0) != 0
    assert call(nV, nT, -1, 0) != 0
    assert call(nV, nT, 12, 5000) != 0
    assert call(nV, nT, 12, 0) == 0 and nt.value == 12
