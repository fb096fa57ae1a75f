"""Pins for the FP64 CPU oracle, against what the paper and the mathematics fix.

None of these compares the oracle with itself:
  * hand-built nets with closed-form zero sets (cube, octahedron, max-pooled
    cube): exact face/vertex/edge counts, area, enclosed volume;
  * the tie rule of the state functional (a unit with pre-activation 0 is off,
    Eqn (NeuronState));
  * the one-hidden-layer special case (the code is the sign pattern of Wx+b);
  * the region-wise linear maps of Lemma 1 / Corollary 1 against a plain
    forward pass at interior points;
  * brute force over every activation code with the paper's naive pair
    enumeration (oracle/brute.py, independent numpy code);
  * Theorem 1 closedness: every edge shared by exactly two faces, Euler
    characteristic 2, and the divergence-theorem volume against Monte Carlo.
"""
import math

import numpy as np
import pytest

import meshcheck as MC
from am_workloads import nets, seeds
from oracle import brute
from oracle import oracle as O


def march_from_ray(net, o=(0.0, 0.0, 0.0), d=(0.9, 0.13, 0.07), lib_path=O.LIB_PATH):
    on = O.OracleNet(net, lib_path)
    st, x, code, am = on.seed_ray(np.asarray(o, float), np.asarray(d, float))
    assert st == 0
    return on, on.march(code[None], np.array([am]))


# ---------------------------------------------------------------- exact nets

@pytest.mark.parametrize("name,F,V,E,area,vol", [
    ("cube", 32, 26, 56, 6.0, 1.0),
    ("octahedron", 8, 6, 12, 4.0 * math.sqrt(3.0) * 0.75 ** 2, (4.0 / 3.0) * 0.75 ** 3),
    ("octahedron_split", 12, 8, 18, 4.0 * math.sqrt(3.0) * 0.75 ** 2, (4.0 / 3.0) * 0.75 ** 3),
    ("maxpool_cube", 6, 8, 12, 6.0, 1.0),
])
def test_exact_nets(name, F, V, E, area, vol):
    net = {"cube": nets.cube_net, "octahedron": nets.octahedron_net,
           "octahedron_split": nets.octahedron_split_net,
           "maxpool_cube": nets.maxpool_cube_net}[name]()
    on, mesh = march_from_ray(net)
    assert mesh.n_faces == F
    assert mesh.stats["degenerate"] == 0
    chi, v, e, f = MC.euler(mesh, net.n_hidden)
    assert (v, e, f, chi) == (V, E, F, 2)
    bad, dom = MC.edge_pairing(mesh, atol=1e-12, n_hidden=net.n_hidden)
    assert bad == 0 and dom == 0
    A, Vol = MC.area_volume(mesh)
    assert abs(A - area) < 1e-12 and abs(Vol - vol) < 1e-12


def test_cube_every_code_is_a_face():
    # Appendix-style derivation: the lines x=0, y=0, y=+-x cut each face of
    # the cube, so all 2^5 activation patterns occur on the surface.
    on, mesh = march_from_ray(nets.cube_net())
    codes = sorted(int(c[0]) for c in mesh.codes)
    assert codes == list(range(32))
    sizes = sorted(np.diff(mesh.offsets))
    assert sizes == [3] * 16 + [4] * 16


def test_maxpool_cube_argmax_states():
    on, mesh = march_from_ray(nets.maxpool_cube_net())
    assert sorted(mesh.argmax.tolist()) == list(range(6))
    # every edge is on a comparison row: ids N + i with N = 0
    assert set(mesh.ids.tolist()) <= set(range(6))


# ------------------------------------------------------------- state / code

def test_code_tie_rule_and_hand_values():
    on = O.OracleNet(nets.cube_net())
    code, am, F = on.code(np.zeros(3))
    assert int(code[0]) == 0 and F == -0.5           # every pre-activation is exactly 0 -> off
    code, am, F = on.code(np.array([0.3, -0.2, 0.1]))
    # u = relu(x,y,z) -> (1,0,1); p = relu(|y|-|x|) off; q = relu(|z|-max) off
    assert int(code[0]) == 0b00101
    assert abs(F - (0.3 - 0.5)) < 1e-15


def test_single_hidden_layer_code_is_sign_pattern():
    net = nets.random_mlp([40], seed=5, bias_std=0.3)
    on = O.OracleNet(net)
    rng = np.random.default_rng(0)
    W1, b1 = net.blocks[0][2], net.bias[0]
    for x in rng.uniform(-1, 1, (50, 3)):
        code, _, _ = on.code(x)
        bits = brute.words_to_bits(code, 40)
        assert bits == tuple(int(v) for v in (W1 @ x + b1 > 0))


def test_forward_matches_numpy_definition():
    net = nets.c1_net()
    on = O.OracleNet(net)
    X = np.random.default_rng(1).uniform(-1, 1, (20, 3))
    ref = brute.forward_pre(net, X)
    for x, r in zip(X, ref):
        F, pre, am = on.forward(x)
        assert np.allclose(pre, r, rtol=1e-13, atol=1e-13)
        assert F == pre[-1]


# ------------------------------------------------------- Lemma 1 identity

@pytest.mark.parametrize("which", ["c1", "maxpool"])
def test_lemma1_identity_at_face_interiors(which):
    if which == "c1":
        net = nets.c1_net()
        on, mesh = march_from_ray(net, d=(1.0, 0.0, 0.0))
    else:
        net = _maxpool_pair([7, 6], [6], 11)
        on = O.OracleNet(net)
        o, d = seeds.random_rays(64, seed=9)
        codes, ams, pts, sts = on.seed_rays(o, d)
        mesh = on.march(codes, ams)
    N = net.n_hidden
    rng = np.random.default_rng(2)
    picks = rng.choice(mesh.n_faces, size=min(200, mesh.n_faces), replace=False)
    worst = 0.0
    for f in picks:
        ids, vs, nb = mesh.face(f)
        w = rng.dirichlet(np.ones(len(vs)))
        x = w @ vs                                      # strictly inside the face
        rows = on.chain(mesh.codes[f])
        F, pre, am = on.forward(x)
        lin = rows @ np.append(x, 1.0)
        scale = 1.0 + np.abs(rows).sum(axis=1)
        worst = max(worst, float(np.max(np.abs(lin - pre) / scale)))
        assert am == mesh.argmax[f]
        assert abs(F) <= 1e-12 * scale[N + am]
        code, am2, _ = on.code(x)
        assert np.array_equal(code, mesh.codes[f])
    assert worst <= 1e-12


# ------------------------------------------------------------ brute force

BRUTE_NETS = (
    [("mlp", [6, 5], s) for s in range(6)]
    + [("sphere", [5, 4], s) for s in range(6)]
    + [("sphere", [9], s) for s in range(3)]
    + [("cube", [4, 4], s) for s in range(4)]
    + [("maxpool", None, s) for s in range(3)]
)


def _centred(net, seed):
    """Shift the head bias so that F changes sign inside the box.

    The shift is the mean of F over random points plus a small offset, so a
    head never ends up exactly 0 on a region where all its units are off.
    """
    X = np.random.default_rng(seed).uniform(-1, 1, (4096, 3))
    med = float(np.mean(brute.forward_pre(net, X)[:, -1])) + 0.0123
    bias = [b.copy() for b in net.bias]
    bias[-1] = bias[-1] - med
    return nets.Net(net.widths, net.blocks, bias)


def _brute_net(kind, hidden, s):
    if kind == "mlp":
        return _centred(nets.random_mlp(hidden, seed=100 + s, bias_std=0.3), s)
    if kind == "sphere":
        return nets.random_sphere_like(hidden, seed=200 + s, radius=0.5, scale=0.4)
    if kind == "cube":
        return nets.shortcut_cube_mlp(hidden, seed=300 + s, scale=0.3)
    return _maxpool_pair([4], [3], s)


def _maxpool_pair(h1, h2, s):
    """Union of two generic random sub-nets (no shared planes), Sec. 5.2."""
    a = _centred(nets.random_mlp(h1, seed=400 + s, bias_std=0.3), s)
    b = _centred(nets.random_mlp(h2, seed=500 + s, bias_std=0.3), s + 1)
    return nets.maxpool_of([a, b])


def _compare_with_brute(net, lib_path=O.LIB_PATH):
    ref = brute.all_faces(net)
    on = O.OracleNet(net, lib_path)
    N = net.n_hidden
    keys = list(ref)
    seed_codes = np.array([brute.bits_to_words(k[0], on.W) for k in keys], np.uint64).reshape(-1, on.W)
    seed_am = np.array([k[1] for k in keys], np.int32)
    mesh = on.march(seed_codes, seed_am)
    got = {}
    for f in range(mesh.n_faces):
        ids, vs, nb = mesh.face(f)
        got[(brute.words_to_bits(mesh.codes[f], N), int(mesh.argmax[f]))] = (ids, vs)
    assert set(got) == set(ref), (len(got), len(ref))
    for k, (ids, vs) in ref.items():
        gi, gv = got[k]
        assert np.array_equal(gi, ids), (k, gi, ids)
        assert np.max(np.abs(gv - vs)) <= 1e-9 * (1.0 + np.abs(vs).max())
    return ref, mesh


@pytest.mark.parametrize("kind,hidden,s", BRUTE_NETS)
def test_march_equals_brute_force(kind, hidden, s):
    net = _brute_net(kind, hidden, s)
    ref, mesh = _compare_with_brute(net)
    assert len(ref) > 0
    # adjacency: a one-seed march reaches exactly the seed's component
    on = O.OracleNet(net)
    k0 = next(iter(ref))
    one = on.march(brute.bits_to_words(k0[0], on.W)[None], np.array([k0[1]], np.int32))
    comp = _component(mesh, k0, net.n_hidden)
    got = {(brute.words_to_bits(one.codes[f], net.n_hidden), int(one.argmax[f])) for f in range(one.n_faces)}
    assert got == comp
    bad, _ = MC.edge_pairing(mesh, n_hidden=net.n_hidden)
    assert bad == 0


def _component(mesh, k0, N):
    keys = [(brute.words_to_bits(mesh.codes[f], N), int(mesh.argmax[f])) for f in range(mesh.n_faces)]
    idx = {k: i for i, k in enumerate(keys)}
    seen = {idx[k0]}
    stack = [idx[k0]]
    while stack:
        f = stack.pop()
        for g in mesh.face(f)[2]:
            if g >= 0 and g not in seen:
                seen.add(int(g))
                stack.append(int(g))
    return {keys[f] for f in seen}


@pytest.mark.slow
@pytest.mark.parametrize("kind,hidden,s", [("mlp", [8, 8], 7), ("cube", [6, 5], 8)])
def test_march_equals_brute_force_16_units(kind, hidden, s):
    net = _brute_net(kind, hidden, s)
    assert net.n_hidden >= 16
    ref, mesh = _compare_with_brute(net)
    assert len(ref) > 0


# ------------------------------------------------------ closedness (C1)

@pytest.fixture(scope="module")
def c1_mesh():
    net = nets.c1_net()
    on, mesh = march_from_ray(net, d=(1.0, 0.0, 0.0))
    return net, on, mesh


def test_c1_closed_genus0(c1_mesh):
    net, on, mesh = c1_mesh
    assert mesh.n_faces > 5000
    assert mesh.stats["degenerate"] == 0 and mesh.stats["seed_empty"] == 0
    bad, dom = MC.edge_pairing(mesh)
    assert bad == 0 and dom == 0
    chi, V, E, F = MC.euler(mesh)
    assert chi == 2


def test_c1_vertices_on_surface_and_feasible(c1_mesh):
    net, on, mesh = c1_mesh
    rng = np.random.default_rng(3)
    for f in rng.choice(mesh.n_faces, 300, replace=False):
        ids, vs, nb = mesh.face(f)
        rows = on.chain(mesh.codes[f])
        N = net.n_hidden
        bits = np.array(brute.words_to_bits(mesh.codes[f], N), float)
        cons = (1.0 - 2.0 * bits)[:, None] * rows[:N]
        for v in vs:
            F, pre, am = on.forward(v)
            assert abs(F) <= 1e-12 * (1.0 + np.abs(rows[N]).sum())
            vals = cons @ np.append(v, 1.0)
            assert np.all(vals <= 1e-11 * (1.0 + np.abs(cons).sum(axis=1)))
            assert np.all(np.abs(v) <= 1.0 + 1e-12)


def test_c1_volume_matches_monte_carlo(c1_mesh):
    net, on, mesh = c1_mesh
    A, Vol = MC.area_volume(mesh)
    rng = np.random.default_rng(4)
    n = 400_000
    X = rng.uniform(-1, 1, (n, 3))
    F = brute.forward_pre(net, X)[:, -1]
    p = float(np.mean(F < 0))
    mc = 8.0 * p
    sigma = 8.0 * math.sqrt(p * (1 - p) / n)
    assert abs(Vol - mc) < 4 * sigma, (Vol, mc, sigma)


# ------------------------------------------------------------- seeding

def test_seed_bisection_lands_on_a_face():
    net = nets.random_sphere_like([6, 5], seed=21, radius=0.5, scale=0.4)
    on = O.OracleNet(net)
    o, d = seeds.random_rays(32, seed=7)
    codes, ams, pts, sts = on.seed_rays(o, d)
    assert (sts == 0).sum() >= 16
    ref = brute.all_faces(net)
    for c, a, x in zip(codes, ams, pts):
        F, pre, am = on.forward(x)
        assert abs(F) <= 1e-12
        assert (brute.words_to_bits(c, net.n_hidden), int(a)) in ref


def test_seed_without_sign_change_is_rejected():
    on = O.OracleNet(nets.cube_net())
    st, x, code, am = on.seed_ray(np.array([0.0, 0.0, 0.0]), np.array([0.2, 0.1, 0.0]))
    assert st == 1


def test_sliver_face_and_zero_area_touch():
    """Which cells count (a face counts iff it has positive area): the sliver
    net's triangle of area 2^-57, about 1 away from the plane's foot point, is
    a face; the cell whose three planes meet in one point of the zero plane
    has a face of zero area and is not one.  Brute force over all 64 codes
    (naive pairs, its own area rule) agrees, and the 14 faces tile the square
    of area 4."""
    net = nets.sliver_net()
    h = 2.0 ** -28
    _compare_with_brute(net)
    on = O.OracleNet(net)
    ids, vs, area, flags = on.face(np.array([0b011011], np.uint64))
    assert area == 2.0 ** -57 and flags == 0
    assert list(ids) == [0, 1, 2]
    want = np.array([[0.75, 0.75 + h, 0.5], [0.75, 0.75, 0.5], [0.75 + h, 0.75, 0.5]])
    for w in want:        # the three corners, in some rotation of the cycle
        assert np.min(np.max(np.abs(vs - w), axis=1)) <= 1e-15
    ids, vs, area, flags = on.face(np.array([0b111000], np.uint64))
    assert len(ids) == 0 and flags & 1
    bits = np.array([0, 0, 0, 1, 1, 1], np.float64)
    rows = brute.chains(net, bits[None])[0]
    assert brute.face_by_pairs(rows, bits, 0, net.n_hidden, net.n_heads) is None
    code, am, _ = on.code(np.array([0.0, 0.0, 0.5]))
    mesh = on.march(code[None], np.array([am]))
    assert mesh.n_faces == 14
    A, _ = MC.area_volume(mesh)
    assert abs(A - 4.0) < 1e-12
