"""Learned form: the proposal scorer, its GPU training kernels, and marches
that clip proposed lines first.

Bars: gradients and Adam steps of the FP32 training kernels vs the FP64
reference (oracle/proposer.py) within 1e-4 relative (norm per tensor); the
FP16 scorer's logits vs the reference on FP16-rounded weights and features
within 5e-3 of max(1, |z|max) (the hidden activations are stored in FP16:
2^-11 relative per value); marches with proposals give exactly the plain
form's cells, cycles and adjacency and its vertices (1e-9; 1e-5 with the
split-BF16 chain); a scorer trained on the GPU accepts more cells than the
method without it.  The training rows come from the GPU clip; they are
inputs of the GPU training only, never of the reference.
"""
import numpy as np
import pytest

from am_workloads import nets, seeds
from gpu_common import compare_meshes_fast, fetch_host, say
from oracle import proposer as RP

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

D, H = 32, 128


@pytest.fixture(scope="module")
def binding():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_10031_amd import binding as B
    return B


def _data(n, seed, used=D):
    rng = np.random.default_rng(seed)
    X = np.zeros((n, D))
    X[:, :used] = rng.normal(0.0, 1.0, (n, used))
    y = (rng.random(n) < 0.2).astype(np.uint8)
    return X.astype(np.float32), y


def _params(seed):
    from paper_2106_10031_amd.learn import init_params
    rng = np.random.default_rng(seed + 100)
    p = init_params(seed).astype(np.float64)
    p += rng.normal(0.0, 0.05, p.shape)          # non-zero biases too
    return p.astype(np.float32)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


@pytest.mark.parametrize("n", [1, 37, 4099])
def test_gradient_matches_fp64_reference(binding, n):
    say("prop grad", n)
    ctx = binding.Context(0)
    X, y = _data(n, seed=n)
    p = _params(1)
    dev = ctx.device
    g = torch.empty(p.size, dtype=torch.float32, device=dev)
    loss = ctx.prop_grad(torch.as_tensor(X, device=dev), torch.as_tensor(y, device=dev),
                         torch.as_tensor(p, device=dev), g)
    ref_loss, ref_g = RP.loss_and_grad(p.astype(np.float64), X.astype(np.float64), y.astype(np.float64), D, H)
    got = g.cpu().numpy().astype(np.float64)
    assert abs(loss - ref_loss) <= 1e-5 * max(1.0, abs(ref_loss))
    o = 0
    for name, size in [("W1", H * D), ("b1", H), ("W2", H * H), ("b2", H), ("w3", H), ("b3", 1)]:
        err = _rel(got[o:o + size], ref_g[o:o + size])
        assert err <= 1e-4, (name, err)
        o += size
    ctx.close()


def test_adam_step_matches_fp64_reference(binding):
    say("prop adam")
    ctx = binding.Context(0)
    rng = np.random.default_rng(7)
    P = ctx.prop_param_count()
    p = rng.normal(size=P).astype(np.float32)
    g = rng.normal(size=P).astype(np.float32)
    m = (0.1 * rng.normal(size=P)).astype(np.float32)
    v = (0.01 * rng.random(P)).astype(np.float32)
    dev = ctx.device
    tp, tg, tm, tv = (torch.as_tensor(a.copy(), device=dev) for a in (p, g, m, v))
    ctx.prop_adam(tp, tg, tm, tv, 3, 1e-3)
    rp, rm, rv = RP.adam_step(p.astype(np.float64), g.astype(np.float64), m.astype(np.float64),
                              v.astype(np.float64), 3, 1e-3)
    assert _rel(tp.cpu().numpy(), rp) <= 1e-6
    assert _rel(tm.cpu().numpy(), rm) <= 1e-6 and _rel(tv.cpu().numpy(), rv) <= 1e-6
    ctx.close()


@pytest.mark.parametrize("n", [5, 64, 1000])
def test_fp16_scorer_matches_reference(binding, n):
    say("prop score", n)
    ctx = binding.Context(0)
    X, _ = _data(n, seed=3 + n, used=8)
    p = _params(2)
    ctx.prop_set(p, k=16, rho=6.0)
    z = ctx.prop_score(torch.as_tensor(X, device=ctx.device)).cpu().numpy()
    q = p.astype(np.float16).astype(np.float64)      # the matrices are stored in FP16
    W1, b1, W2, b2, w3, b3 = RP.unpack(p.astype(np.float64), D, H)
    qW1, _, qW2, _, _, _ = RP.unpack(q, D, H)
    ref = RP.logits(RP.pack(qW1, b1, qW2, b2, w3, np.float32(b3)), X.astype(np.float16).astype(np.float64), D, H)
    assert np.max(np.abs(z - ref)) <= 5e-3 * max(1.0, np.abs(ref).max()), np.max(np.abs(z - ref))
    ctx.close()


def _march(ctx, o, d, **kw):
    ctx.seed_rays(o, d)
    st = ctx.march(max_cells=1 << 21, **kw)
    return st, fetch_host(ctx)


def _c2():
    net = nets.load_fitted("c2")
    prim = np.load(nets.DATA_DIR + "/c2_primitives.npz")
    o, d = seeds.centre_rays(prim["p0"], 128)
    return net, o, d


@pytest.fixture(scope="module")
def trained(binding):
    """A scorer trained on the GPU on rows from the C1 net and the 6x90 fit."""
    from paper_2106_10031_amd import learn
    Xs, ys = [], []
    for net, (o, d) in [(nets.c1_net(), seeds.random_rays(64, seed=11)), (_c2()[0], _c2()[1:])]:
        ctx = binding.Context(0).load_net(net)
        X, y = learn.collect(ctx, o, d, cap=1 << 20)
        Xs.append(X.clone())
        ys.append(y.clone())
        ctx.close()
    X = torch.cat(Xs)
    y = torch.cat(ys)
    ctx = binding.Context(0)
    say("train scorer on", X.shape[0], "rows, positive rate", float(y.float().mean()))
    p, losses = learn.train(ctx, X, y, steps=150, lr=3e-3)
    ctx.close()
    return p, losses, float(y.float().mean())


def test_training_lowers_the_loss(trained):
    p, losses, pos = trained
    base = -(pos * np.log(pos) + (1 - pos) * np.log(1 - pos))     # loss of the label rate alone
    say(f"loss {losses[0]:.4f} -> {losses[-1]:.4f} (label-rate entropy {base:.4f})")
    assert np.all(np.isfinite(p))
    assert losses[-1] < 0.6 * base


@pytest.mark.parametrize("propose", [1, 2])
def test_proposals_leave_the_mesh_unchanged(binding, trained, propose):
    net, o, d = _c2()
    say("c2 plain vs propose", propose)
    ctx = binding.Context(0).load_net(net)
    ctx.prop_set(trained[0], k=16, rho=6.0)
    st0, ref = _march(ctx, o, d)
    st1, got = _march(ctx, o, d, propose=propose)
    assert st1["faces"] == st0["faces"] == 471884
    compare_meshes_fast(ref, got, vtol=1e-9)
    ctx.close()


def test_learned_bf16_form_matches_fp64(binding, trained):
    net, o, d = _c2()
    say("c2 plain FP64 vs learned + split-BF16")
    ctx = binding.Context(0).load_net(net)
    ctx.prop_set(trained[0], k=16, rho=6.0)
    _, ref = _march(ctx, o, d)
    _, got = _march(ctx, o, d, propose=1, precision=1)
    compare_meshes_fast(ref, got, vtol=1e-5)
    ctx.close()


def test_trained_scorer_accepts_more_cells(binding, trained):
    net, o, d = _c2()
    ctx = binding.Context(0).load_net(net)
    ctx.prop_set(trained[0], k=16, rho=6.0)
    rates = {}
    for mode, name in [(3, "none"), (2, "distance"), (1, "learned")]:
        st, _ = _march(ctx, o, d, propose=mode)
        rates[name] = (st["prop_accepted"] / st["prop_cells"], st["prop_cuts"] / st["prop_cells"])
    say("accept rate / cuts per cell in the every-line pass:",
        {k: (round(a, 4), round(c, 3)) for k, (a, c) in rates.items()})
    assert rates["learned"][0] > rates["none"][0]
    assert rates["learned"][1] < rates["none"][1]
    ctx.close()
