"""GPU parity: every stage of the HIP path, called through the C-ABI, against the oracle.

Bar: activation codes, cell sets, polygon id cycles and adjacency bit-exact;
affine rows within 1e-12 relative; vertices within 1e-9 relative
(|dv|_inf / max(1, |v|_inf)) on the FP64 path.
"""
import numpy as np
import pytest

import meshcheck as MC
from am_workloads import nets, seeds
from gpu_common import compare_meshes, fetch_host, say
from oracle import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def binding():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_10031_amd import binding as B
    return B


def _ctx(B, net):
    return B.Context(0).load_net(net)


def _oracle_mesh(net, o, d):
    on = O.OracleNet(net)
    codes, ams, pts, sts = on.seed_rays(o, d)
    return on, on.march(codes, ams)


SMALL_NETS = {
    "cube": nets.cube_net,
    "octahedron_split": nets.octahedron_split_net,
    "maxpool_cube": nets.maxpool_cube_net,
    "c1": nets.c1_net,
    "sphere_like_2x24": lambda: nets.random_sphere_like([24, 24], seed=5, radius=0.6, scale=0.4),
}


# ------------------------------------------------------------------ stages

@pytest.mark.parametrize("name", ["c1", "sphere_like_2x24", "maxpool_cube"])
def test_codes_match_oracle(binding, name):
    net = SMALL_NETS[name]()
    say("codes", name)
    ctx = _ctx(binding, net)
    X = np.random.default_rng(0).uniform(-1, 1, (257, 3))
    X[0] = 0.0                                # ties: every unit of the cube part is exactly 0
    codes, am, F = ctx.codes(X)
    torch.cuda.synchronize()
    on = O.OracleNet(net)
    codes = codes.cpu().numpy().view(np.uint64)
    am = am.cpu().numpy()
    F = F.cpu().numpy()
    for i, x in enumerate(X):
        c, a, f = on.code(x)
        assert np.array_equal(codes[i], c), i
        assert am[i] == a
        assert abs(F[i] - f) <= 1e-12 * (1 + abs(f))


@pytest.mark.parametrize("name", ["c1", "sphere_like_2x24", "octahedron_split"])
def test_chain_matches_oracle(binding, name):
    net = SMALL_NETS[name]()
    on, mesh = _oracle_mesh(net, *seeds.random_rays(8, seed=1))
    pick = np.random.default_rng(1).choice(mesh.n_faces, size=min(333, mesh.n_faces), replace=False)
    codes = mesh.codes[pick]
    say("chain", name, len(pick))
    ctx = _ctx(binding, net)
    rows = ctx.chain(torch.as_tensor(codes.view(np.int64)).cuda())
    torch.cuda.synchronize()
    rows = rows.cpu().numpy()
    for i, c in enumerate(codes):
        ref = on.chain(c)
        scale = 1.0 + np.abs(ref).sum(axis=1, keepdims=True)
        assert np.max(np.abs(rows[i] - ref) / scale) <= 1e-12


@pytest.mark.parametrize("name", ["c1", "sphere_like_2x24", "octahedron_split", "maxpool_cube"])
def test_faces_match_oracle(binding, name):
    net = SMALL_NETS[name]()
    on, mesh = _oracle_mesh(net, *seeds.random_rays(8, seed=2))
    say("faces", name, mesh.n_faces)
    ctx = _ctx(binding, net)
    m, ids, verts, flags = ctx.faces(torch.as_tensor(mesh.codes.view(np.int64)).cuda(),
                                     torch.as_tensor(mesh.argmax).cuda(), max_m=48)
    torch.cuda.synchronize()
    m, ids, verts, flags = (t.cpu().numpy() for t in (m, ids, verts, flags))
    for f in range(mesh.n_faces):
        rid, rv, _ = mesh.face(f)
        assert m[f] == len(rid), f
        assert np.array_equal(ids[f, :m[f]], rid), (f, ids[f, :m[f]], rid)
        assert np.max(np.abs(verts[f, :m[f]] - rv)) <= 1e-9 * max(1.0, np.abs(rv).max())


def test_seed_rays_match_oracle(binding):
    net = SMALL_NETS["sphere_like_2x24"]()
    o, d = seeds.random_rays(96, seed=3)
    say("seed_rays", len(o))
    ctx = _ctx(binding, net)
    status = ctx.seed_rays(o, d)
    torch.cuda.synchronize()
    status = status.cpu().numpy()
    on = O.OracleNet(net)
    for i in range(len(o)):
        st, x, code, am = on.seed_ray(o[i], d[i])
        assert status[i] == st, i
    # the seeds' cells, as marched, contain the oracle's seed cells
    st = ctx.march()
    got = fetch_host(ctx)
    codes, ams, pts, sts = on.seed_rays(o, d)
    have = {MC.code_key(got.codes[f], got.argmax[f]) for f in range(got.n_faces)}
    for c, a in zip(codes, ams):
        assert MC.code_key(c, a) in have


# ------------------------------------------------------------------ march

@pytest.mark.parametrize("path", [1, 2], ids=["split", "fused"])
@pytest.mark.parametrize("name", list(SMALL_NETS))
def test_march_matches_oracle(binding, name, path):
    net = SMALL_NETS[name]()
    o, d = seeds.random_rays(16, seed=4)
    on, ref = _oracle_mesh(net, o, d)
    say("march", name, ref.n_faces, "path", path)
    ctx = _ctx(binding, net)
    ctx.seed_rays(o, d)
    st = ctx.march(kernel_path=path)
    assert st["fused"] == (path == 2)
    got = fetch_host(ctx)
    assert st["faces"] == ref.n_faces
    assert st["cells"] == ref.stats["cells"]
    compare_meshes(ref, got)
    bad, dom = MC.edge_pairing(got, n_hidden=net.n_hidden)
    assert bad == 0


def test_march_c1_axis_seed(binding):
    net = nets.c1_net()
    o, d = seeds.axis_ray()
    on, ref = _oracle_mesh(net, o, d)
    say("march c1 +x seed", ref.n_faces)
    ctx = _ctx(binding, net)
    ctx.seed_rays(o, d)
    st = ctx.march()
    got = fetch_host(ctx)
    compare_meshes(ref, got)
    assert MC.euler(got, net.n_hidden)[0] == 2
    assert st["domain_edges"] == 0 and st["degenerate"] == 0


def test_march_is_deterministic_as_a_set(binding):
    net = nets.c1_net()
    o, d = seeds.random_rays(64, seed=5)
    say("march twice", "c1")
    ctx = _ctx(binding, net)
    ctx.seed_rays(o, d)
    ctx.march()
    a = MC.by_code(fetch_host(ctx))
    ctx.seed_rays(o, d)
    ctx.march()
    b = MC.by_code(fetch_host(ctx))
    assert set(a) == set(b)
    for k in a:
        assert np.array_equal(a[k][0], b[k][0]) and a[k][2] == b[k][2]
        assert np.array_equal(a[k][1], b[k][1])


# ------------------------------------------------------------- edge cases

def test_capacity_error_then_retry(binding):
    net = nets.c1_net()
    o, d = seeds.axis_ray()
    say("capacity", "c1")
    ctx = _ctx(binding, net)
    ctx.seed_rays(o, d)
    with pytest.raises(binding.AmError) as e:
        ctx.march(max_cells=1000)
    assert e.value.status == binding.AM_E_CAPACITY
    assert e.value.stats["required_cells"] > 1000
    st = ctx.march(max_cells=1 << 16)
    assert st["faces"] > 1000


def test_invalid_inputs_are_rejected(binding):
    say("invalid inputs")
    net = nets.cube_net()
    bad = nets.Net(net.widths, [(d, s, W.copy()) for d, s, W in net.blocks], [b.copy() for b in net.bias])
    bad.blocks[0][2][0, 0] = np.nan
    ctx = binding.Context(0)
    with pytest.raises(binding.AmError) as e:
        ctx.load_net(bad)
    assert e.value.status == binding.AM_E_INVALID
    with pytest.raises(binding.AmError) as e:
        ctx.march()
    assert e.value.status == binding.AM_E_STATE
    ctx.load_net(net)
    # a ray without a sign change gives no seed
    ctx.seed_rays(np.zeros((1, 3)), np.array([[0.2, 0.1, 0.0]]))
    with pytest.raises(binding.AmError) as e:
        ctx.march()
    assert e.value.status == binding.AM_E_SEED


def test_empty_seed_cell_is_reported(binding):
    say("empty seed cell")
    net = nets.cube_net()
    ctx = _ctx(binding, net)
    # code 0b00101 with argmax 0 has a face; an out-of-range argmax does not seed
    codes = torch.tensor([[0b00101]], dtype=torch.int64).cuda()
    ctx.seed_cells(codes, torch.tensor([0], dtype=torch.int32).cuda())
    st = ctx.march()
    assert st["faces"] == 32


# ------------------------------------------- full-size workload (bench's)

@pytest.fixture(scope="module")
def c2_case():
    from am_workloads import nets as N
    net = N.load_fitted("c2")
    prim = np.load(__import__("os").path.join(N.DATA_DIR, "c2_primitives.npz"))
    o, d = seeds.centre_rays(prim["p0"], 128)
    return net, o, d


def test_c2_full_march_sampled_faces_and_closedness(binding, c2_case):
    """The bench workload at full size: sampled faces one by one + invariants."""
    net, o, d = c2_case
    say("c2 full march (sampled)")
    ctx = _ctx(binding, net)
    ctx.seed_rays(o, d)
    st = ctx.march(max_cells=1 << 21)
    got = fetch_host(ctx)
    assert st["faces"] == got.n_faces and st["degenerate"] == 0
    on = O.OracleNet(net)
    rng = np.random.default_rng(7)
    for f in rng.choice(got.n_faces, 2000, replace=False):
        ids, vs, nb = got.face(f)
        rid, rv, _, fl = on.face(got.codes[f], got.argmax[f])
        assert fl == 0 and np.array_equal(ids, rid)
        assert np.max(np.abs(vs - rv)) <= 1e-9 * max(1.0, np.abs(rv).max())
    bad, dom = MC.edge_pairing(got, n_hidden=net.n_hidden)
    assert bad == 0
    # every seed the oracle finds is a marched cell
    codes, ams, _, _ = on.seed_rays(o, d)
    have = {MC.code_key(got.codes[f], got.argmax[f]) for f in range(got.n_faces)}
    assert all(MC.code_key(c, a) in have for c, a in zip(codes, ams))


@pytest.fixture(scope="module")
def c2_ref(c2_case):
    net, o, d = c2_case
    on = O.OracleNet(net)
    codes, ams, _, _ = on.seed_rays(o, d)
    return on.march(codes, ams)


@pytest.mark.parametrize("path", [1, 0], ids=["split", "auto"])
def test_c2_full_march_equals_oracle(binding, c2_case, c2_ref, path):
    """The whole cell set, cycles and adjacency against the oracle's full march."""
    net, o, d = c2_case
    ref = c2_ref
    say("c2 full march vs oracle", ref.n_faces, "path", path)
    ctx = _ctx(binding, net)
    ctx.seed_rays(o, d)
    st = ctx.march(max_cells=1 << 21, kernel_path=path)
    got = fetch_host(ctx)
    assert st["faces"] == ref.n_faces and st["cells"] == ref.stats["cells"]
    compare_meshes(ref, got)


# ------------------------------------------------------- canonical fetch

def _fetch_sorted_host(ctx):
    from paper_2106_10031_amd.binding import mesh_to_host
    from gpu_common import HostMesh
    h = mesh_to_host(ctx.fetch(sorted=True))
    return HostMesh(h["codes"], h["argmax"], h["offsets"], h["ids"], h["verts"], h["nbr"]), h["shape"]


def _assert_arrays_equal_oracle(ref, got, vtol=1e-9):
    assert np.array_equal(got.offsets, ref.offsets)
    assert np.array_equal(got.codes, ref.codes) and np.array_equal(got.argmax, ref.argmax)
    assert np.array_equal(got.ids, ref.ids)
    assert np.array_equal(got.nbr, ref.nbr)
    scale = np.maximum(1.0, np.abs(ref.verts).max(axis=1))
    assert (np.abs(got.verts - ref.verts).max(axis=1) / scale).max() <= vtol


@pytest.mark.parametrize("name", list(SMALL_NETS))
def test_fetch_sorted_equals_oracle_arrays(binding, name):
    """am_fetch_sorted gives the oracle's canonical mesh array for array."""
    net = SMALL_NETS[name]()
    o, d = seeds.random_rays(16, seed=4)
    on, ref = _oracle_mesh(net, o, d)
    say("fetch sorted", name, ref.n_faces)
    ctx = _ctx(binding, net)
    ctx.seed_rays(o, d)
    ctx.march()
    got, _ = _fetch_sorted_host(ctx)
    _assert_arrays_equal_oracle(ref, got)


def test_fetch_sorted_c2_equals_oracle_arrays(binding, c2_case, c2_ref):
    net, o, d = c2_case
    say("fetch sorted c2", c2_ref.n_faces)
    ctx = _ctx(binding, net)
    ctx.seed_rays(o, d)
    ctx.march(max_cells=1 << 21)
    got, _ = _fetch_sorted_host(ctx)
    _assert_arrays_equal_oracle(c2_ref, got)


def test_fetch_sorted_batched_orders_by_shape(binding):
    sb = nets.latent_sphere_batch([16, 16, 16], reinject=3, latent_dim=8, n_shapes=6, seed=3)
    o, d, sh = [], [], []
    for s in range(sb.n_shapes):
        a, b = seeds.random_rays(12, seed=100 + s)
        o.append(a); d.append(b); sh.append(np.full(12, s, np.int32))
    o, d, sh = np.concatenate(o), np.concatenate(d), np.concatenate(sh)
    say("fetch sorted batched")
    ctx = binding.Context(0).load_net(sb.net, shape_bias=sb.shape_bias)
    ctx.seed_rays(o, d, shape_id=sh)
    ctx.march()
    from paper_2106_10031_amd.binding import mesh_to_host
    plain = mesh_to_host(ctx.fetch())
    got, shape = _fetch_sorted_host(ctx)
    keys = [(int(shape[f]),) + tuple(int(w) for w in got.codes[f]) + (int(got.argmax[f]),)
            for f in range(got.n_faces)]
    assert all(a < b for a, b in zip(keys, keys[1:]))
    # the host's own ordering of the discovery-order fetch, neighbours remapped
    codes = plain["codes"]
    order = np.lexsort([plain["argmax"]] + [codes[:, w] for w in range(codes.shape[1] - 1, -1, -1)]
                       + [plain["shape"]])
    inv = np.empty_like(order)
    inv[order] = np.arange(len(order))
    off = plain["offsets"]
    ms = np.diff(off)[order]
    idx = np.concatenate([np.arange(off[f], off[f + 1]) for f in order])
    nb = plain["nbr"][idx]
    nb = np.where(nb >= 0, inv[np.maximum(nb, 0)], nb)
    assert np.array_equal(np.diff(got.offsets), ms)
    assert np.array_equal(got.ids, plain["ids"][idx]) and np.array_equal(got.verts, plain["verts"][idx])
    assert np.array_equal(got.nbr, nb)
    assert np.array_equal(shape, plain["shape"][order])
    ctx.close()


def test_seed_points_march_matches_oracle(binding):
    """am_seed_points: seeds are the cells of the given points; surface points
    from the oracle's own ray seeding give the oracle's mesh, and an
    off-surface point adds no face."""
    net = nets.c1_net()
    o, d = seeds.random_rays(16, seed=4)
    on = O.OracleNet(net)
    codes, ams, pts, sts = on.seed_rays(o, d)
    ref = on.march(codes, ams)
    say("seed points c1", len(pts))
    ctx = _ctx(binding, net)
    far = np.array([[0.0, 0.0, 0.0]])            # F(0) < 0: inside, its cell has no face
    ctx.seed_points(np.vstack([pts[sts == 0], far]))
    st = ctx.march()
    assert st["faces"] == ref.n_faces
    compare_meshes(ref, fetch_host(ctx))
    ctx.seed_points(far)
    with pytest.raises(binding.AmError) as e:
        ctx.march()
    assert "AM_E_SEED" in str(e.value)
