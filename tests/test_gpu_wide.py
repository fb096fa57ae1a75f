"""The wide workloads at full size: the 64-shape 8x512 decoder batch and the
3->[512]x8->1 sphere-union fit (39 M faces).

Bars:
* batched form: every shape's part of one batched march equals its own
  single-shape march array for array (cells, cycles, adjacency exact,
  vertices bit-equal: same rows, same solves), on all 64 shapes;
* sampled faces of both workloads equal the oracle's faces of the same cells
  (cycles exact, vertices 1e-9 relative), over the whole box-size range for
  the batch and >= 10,000 faces of the 8x512 fit;
* closedness (Theorem 1) of the whole 8x512 mesh: across every inner edge on
  unit k the neighbour's edge on unit k points back;
* the three patterns together (split-BF16 chain, proposals, batching) on all
  64 shapes at the default certificate: the plain batched mesh's cells,
  cycles and adjacency, vertices within 1e-5.

Whole-mesh comparisons run on the device (torch): the meshes are fetched in
canonical order (shape, code words, argmax), so shape s of a batched march
is one contiguous block that a single-shape march of s reproduces.
"""
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


def test_c5_sampled_faces_and_closedness(binding):
    net = nets.load_fitted("c5")
    prim = np.load(nets.DATA_DIR + "/c5_primitives.npz")
    o, d = seeds.centre_rays(prim["p0"], 128)
    say("c5: full march")
    ctx = binding.Context(0).load_net(net)
    ctx.seed_rays(o, d)
    st = ctx.march(max_cells=1 << 26)
    out = ctx.fetch(sorted=True)
    torch.cuda.synchronize()
    F = st["faces"]
    assert st["degenerate"] == 0
    # closedness: the edge (face f, unit k) with neighbour g has a twin (g, k)
    # whose neighbour is f
    off = out["offsets"]
    ms = off[1:] - off[:-1]
    face_of = torch.repeat_interleave(torch.arange(F, device=off.device), ms)
    ids = out["ids"].to(torch.int64)
    nbr = out["nbr"]
    K = net.n_hidden + net.n_heads + 8
    keys = face_of * K + (ids + 7)
    order = torch.argsort(keys)
    sk = keys[order]
    inner = nbr >= 0
    want = nbr[inner] * K + (ids[inner] + 7)
    pos = torch.searchsorted(sk, want).clamp(max=sk.numel() - 1)
    assert torch.equal(sk[pos], want), "an inner edge has no twin"
    assert torch.equal(nbr[order][pos], face_of[inner]), "a twin does not point back"
    say("c5 closed:", F, "faces,", int(inner.sum().item()), "inner edges")
    # >= 10,000 sampled faces against the oracle
    rng = np.random.default_rng(17)
    fs = np.sort(rng.choice(F, size=10240, replace=False))
    fs_d = torch.as_tensor(fs, device=off.device)
    codes = out["codes"][fs_d].cpu().numpy().view(np.uint64)
    am = out["argmax"][fs_d].cpu().numpy()
    on = O.OracleNet(net, lib_path=O.OMP_LIB_PATH)
    m, rid, rv, flags = on.faces_batched(codes, am)
    offh = off.cpu().numpy()
    idsh = out["ids"].cpu().numpy()
    vh = out["verts"].cpu().numpy()
    worst = 0.0
    for i, f in enumerate(fs):
        lo, hi = offh[f], offh[f + 1]
        assert flags[i] == 0 and m[i] == hi - lo, f
        assert np.array_equal(idsh[lo:hi], rid[i, :m[i]]), f
        r = rv[i, :m[i]]
        worst = max(worst, float(np.max(np.abs(vh[lo:hi] - r)) / max(1.0, np.abs(r).max())))
    assert worst <= 1e-9, worst
    say("c5 oracle faces checked", len(fs), "worst vertex error", worst)
    ctx.close()
    del out, keys, order, sk
    torch.cuda.empty_cache()


def c4_rays():
    sb = nets.c4_batch()
    o, d, sh = nets.c4_seed_rays(sb.n_shapes)
    return sb, o, d, sh


@pytest.fixture(scope="module")
def c4_batched(binding):
    """The plain batched march of all 64 shapes, fetched in canonical order."""
    sb, o, d, sh = c4_rays()
    say("c4: batched march of 64 shapes")
    ctx = binding.Context(0).load_net(sb.net, shape_bias=sb.shape_bias)
    ctx.seed_rays(o, d, shape_id=sh)
    st = ctx.march(max_cells=1 << 24)
    out = ctx.fetch(sorted=True)
    torch.cuda.synchronize()
    yield sb, ctx, st, out
    ctx.close()


def shape_blocks(out, S):
    """Face and corner ranges of each shape in a canonical fetch."""
    shape = out["shape"]
    f_lo = torch.searchsorted(shape, torch.arange(S + 1, dtype=shape.dtype, device=shape.device)).cpu().numpy()
    off = out["offsets"].cpu().numpy()
    return f_lo, off[f_lo]


def test_c4_batched_equals_all_64_single_shape_marches(binding, c4_batched):
    sb, ctx, st, out = c4_batched
    _, o, d, sh = c4_rays()
    S = sb.n_shapes
    f_lo, c_lo = shape_blocks(out, S)
    total = 0
    for s in range(S):
        m = sh == s
        ctx.seed_rays(o[m], d[m], shape_id=sh[m])
        one_st = ctx.march(max_cells=1 << 24)
        one = ctx.fetch(sorted=True)
        a, b = int(f_lo[s]), int(f_lo[s + 1])
        ca, cb = int(c_lo[s]), int(c_lo[s + 1])
        assert one_st["faces"] == b - a, (s, one_st["faces"], b - a)
        assert torch.equal(one["codes"], out["codes"][a:b]), s
        assert torch.equal(one["argmax"], out["argmax"][a:b]), s
        assert torch.all(out["shape"][a:b] == s)
        assert torch.equal(one["offsets"], out["offsets"][a:b + 1] - ca), s
        assert torch.equal(one["ids"], out["ids"][ca:cb]), s
        nb = out["nbr"][ca:cb]
        assert torch.equal(one["nbr"], torch.where(nb >= 0, nb - a, nb)), s
        assert torch.equal(one["verts"], out["verts"][ca:cb]), s
        total += b - a
    assert total == st["faces"]
    counts = np.diff(f_lo)
    say("c4 faces per shape", int(counts.min()), "..", int(counts.max()))


def test_c4_sampled_faces_equal_the_oracle_across_box_sizes(binding, c4_batched):
    sb, ctx, st, out = c4_batched
    S = sb.n_shapes
    f_lo, _ = shape_blocks(out, S)
    rng = np.random.default_rng(13)
    off = out["offsets"].cpu().numpy()
    checked = 0
    for s in (0, 9, 18, 27, 36, 45, 54, 63):           # box half-sizes 1.2e-3 ... 0.125
        a, b = int(f_lo[s]), int(f_lo[s + 1])
        fs = rng.choice(np.arange(a, b), size=min(150, b - a), replace=False)
        codes = out["codes"][torch.as_tensor(fs, device=out["codes"].device)].cpu().numpy().view(np.uint64)
        am = out["argmax"][torch.as_tensor(fs, device=out["codes"].device)].cpu().numpy()
        on = O.OracleNet(sb.shape_net(s), lib_path=O.OMP_LIB_PATH)
        m, ids, verts, flags = on.faces_batched(codes, am)
        for i, f in enumerate(fs):
            lo, hi = off[f], off[f + 1]
            assert flags[i] == 0 and m[i] == hi - lo, (s, f)
            assert np.array_equal(out["ids"][lo:hi].cpu().numpy(), ids[i, :m[i]]), (s, f)
            gv = out["verts"][lo:hi].cpu().numpy()
            rv = verts[i, :m[i]]
            assert np.max(np.abs(gv - rv)) <= 1e-9 * max(1.0, np.abs(rv).max()), (s, f)
        checked += len(fs)
    say("c4 oracle faces checked", checked)


def test_c4_split_bf16_with_proposals_default_certificate(binding, c4_batched):
    """All 64 shapes, split-BF16 chain and distance-ordered proposals together,
    default vertex_tol (1e-5) and the certificate measured for this decoder."""
    sb, ctx, st, out = c4_batched
    _, o, d, sh = c4_rays()
    say("c4: split-BF16 + proposals, batched, default certificate")
    ctx.seed_rays(o, d, shape_id=sh)
    st2 = ctx.march(max_cells=1 << 24, precision=1, propose=2)
    got = ctx.fetch(sorted=True)
    assert st2["faces"] == st["faces"]
    for k in ("codes", "argmax", "shape", "offsets", "ids", "nbr"):
        assert torch.equal(got[k], out[k]), k
    rv = out["verts"]
    err = ((got["verts"] - rv).abs().amax(dim=1) / rv.abs().amax(dim=1).clamp(min=1.0)).max().item()
    say("c4 split-bf16: max vertex error", err, "escalated", st2["escalated"], "of", st2["cells"],
        "row eps", st2["split_row_eps"], "margin", st2["split_margin"], "measured on", st2["calib_vertices"])
    assert err <= 1e-5
    assert st2["split_row_eps"] > 0 and st2["calib_vertices"] > 0
