"""Network descriptions and seeded network generators.

This module only *describes* inputs: layer widths, dense weight blocks and
biases.  It holds none of the meshing arithmetic; both the GPU library and the
CPU oracle consume the same :class:`Net` through their own bindings.

Layout of a net (a DAG of dense blocks, covering plain MLPs, identity and
linear shortcuts, and max-pooled heads; Sec. 2.2, Sec. 5.1 and Sec. 5.2 of the
paper):

* layer 0 is the input ``x`` in R^3 (never rectified);
* layers 1..L are hidden ReLU layers;
* layer L+1 holds the M >= 1 output heads; the implicit function is
  ``F(x) = max_i head_i(x)`` (M = 1 is a plain regressor);
* every block ``(dst, src, W)`` with ``src < dst`` adds ``W @ act[src]`` to the
  pre-activation of layer ``dst``; ``act[0] = x`` and ``act[l] = relu(pre[l])``.
"""
from __future__ import annotations

import dataclasses
import hashlib
import os
from typing import List, Sequence, Tuple

import numpy as np

DATA_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data")


@dataclasses.dataclass
class Net:
    widths: List[int]                              # [3, n_1, ..., n_L, M]
    blocks: List[Tuple[int, int, np.ndarray]]      # (dst, src, W[n_dst, n_src])
    bias: List[np.ndarray]                         # bias[l-1] for l = 1..L+1

    def __post_init__(self):
        self.widths = [int(w) for w in self.widths]
        self.blocks = [(int(d), int(s), np.ascontiguousarray(W, dtype=np.float64))
                       for d, s, W in self.blocks]
        self.bias = [np.ascontiguousarray(b, dtype=np.float64).reshape(-1) for b in self.bias]
        self.blocks.sort(key=lambda t: (t[0], t[1]))
        self.validate()

    # ---- shape helpers -------------------------------------------------
    @property
    def n_hidden_layers(self) -> int:
        return len(self.widths) - 2

    @property
    def n_hidden(self) -> int:
        """N: total number of hidden ReLU units (the code length)."""
        return int(sum(self.widths[1:-1]))

    @property
    def n_heads(self) -> int:
        return self.widths[-1]

    def validate(self):
        w = self.widths
        if len(w) < 2 or w[0] != 3 or w[-1] < 1 or any(x < 1 for x in w[1:]):
            raise ValueError(f"bad widths {w}")
        if len(self.bias) != len(w) - 1:
            raise ValueError("need one bias vector per non-input layer")
        for l, b in enumerate(self.bias, start=1):
            if b.shape != (w[l],):
                raise ValueError(f"bias of layer {l} has shape {b.shape}")
        seen = set()
        for d, s, W in self.blocks:
            if not (0 <= s < d < len(w)):
                raise ValueError(f"block {d}<-{s} is not feed-forward")
            if (d, s) in seen:
                raise ValueError(f"duplicate block {d}<-{s}")
            seen.add((d, s))
            if W.shape != (w[d], w[s]):
                raise ValueError(f"block {d}<-{s} has shape {W.shape}, want {(w[d], w[s])}")
        for l in range(1, len(w)):
            if not any(d == l for d, _, _ in self.blocks):
                raise ValueError(f"layer {l} has no input block")

    def astype(self, dtype) -> "Net":
        """A copy with every parameter rounded to ``dtype`` (then held in float64)."""
        return Net(list(self.widths),
                   [(d, s, W.astype(dtype).astype(np.float64)) for d, s, W in self.blocks],
                   [b.astype(dtype).astype(np.float64) for b in self.bias])

    def digest(self) -> str:
        h = hashlib.sha256()
        h.update(np.asarray(self.widths, np.int64).tobytes())
        for d, s, W in self.blocks:
            h.update(np.asarray([d, s], np.int64).tobytes())
            h.update(W.tobytes())
        for b in self.bias:
            h.update(b.tobytes())
        return h.hexdigest()

    # ---- persistence (plain arrays, no pickles) -------------------------
    def save(self, path: str, dtype=np.float64):
        arrs = {"widths": np.asarray(self.widths, np.int64),
                "block_ds": np.asarray([[d, s] for d, s, _ in self.blocks], np.int64)}
        for i, (_, _, W) in enumerate(self.blocks):
            arrs[f"W{i}"] = W.astype(dtype)
        for l, b in enumerate(self.bias, start=1):
            arrs[f"b{l}"] = b.astype(dtype)
        np.savez(path, **arrs)

    @staticmethod
    def load(path: str) -> "Net":
        z = np.load(path, allow_pickle=False)
        widths = [int(v) for v in z["widths"]]
        ds = z["block_ds"]
        blocks = [(int(ds[i, 0]), int(ds[i, 1]), z[f"W{i}"].astype(np.float64))
                  for i in range(ds.shape[0])]
        bias = [z[f"b{l}"].astype(np.float64) for l in range(1, len(widths))]
        return Net(widths, blocks, bias)


# ---------------------------------------------------------------------------
# Hand-built exact nets (all weights dyadic, so every row is exact in FP64).
# ---------------------------------------------------------------------------

def cube_net() -> Net:
    """g(x) = max(|x|,|y|,|z|) - 0.5: the zero set is the cube [-0.5,0.5]^3.

    Units: layer 1 u = relu(x), relu(y), relu(z); layer 2 p = relu(|y| - |x|);
    layer 3 q = relu(|z| - max(|x|,|y|)); head g = |x| + p + q - 0.5 with
    |t| = 2 relu(t) - t.  Identity/linear shortcuts as in Sec. 5.1.
    """
    widths = [3, 3, 1, 1, 1]
    blocks = [
        (1, 0, np.eye(3)),
        (2, 1, np.array([[-2.0, 2.0, 0.0]])),
        (2, 0, np.array([[1.0, -1.0, 0.0]])),
        (3, 1, np.array([[-2.0, 0.0, 2.0]])),
        (3, 0, np.array([[1.0, 0.0, -1.0]])),
        (3, 2, np.array([[-1.0]])),
        (4, 1, np.array([[2.0, 0.0, 0.0]])),
        (4, 0, np.array([[-1.0, 0.0, 0.0]])),
        (4, 2, np.array([[1.0]])),
        (4, 3, np.array([[1.0]])),
    ]
    bias = [np.zeros(3), np.zeros(1), np.zeros(1), np.array([-0.5])]
    return Net(widths, blocks, bias)


def octahedron_net(r: float = 0.75) -> Net:
    """|x| + |y| + |z| - r with |t| = 2 relu(t) - t (one hidden layer of 3)."""
    widths = [3, 3, 1]
    blocks = [(1, 0, np.eye(3)),
              (2, 1, np.array([[2.0, 2.0, 2.0]])),
              (2, 0, np.array([[-1.0, -1.0, -1.0]]))]
    bias = [np.zeros(3), np.array([-r])]
    return Net(widths, blocks, bias)


def octahedron_split_net(r: float = 0.75) -> Net:
    """The octahedron net plus a unit relu(x + y) that the head ignores.

    The plane x + y = 0 cuts the four faces with sign(x) != sign(y) in two and
    passes exactly through the apexes (0, 0, +-r), where it only touches the
    other four faces: F = 12, V = 8, E = 18, area and volume unchanged.
    """
    widths = [3, 4, 1]
    W1 = np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0], [1.0, 1.0, 0.0]])
    blocks = [(1, 0, W1),
              (2, 1, np.array([[2.0, 2.0, 2.0, 0.0]])),
              (2, 0, np.array([[-1.0, -1.0, -1.0]]))]
    bias = [np.zeros(4), np.array([-r])]
    return Net(widths, blocks, bias)


def maxpool_cube_net() -> Net:
    """F = max_i (+-x_i - 0.5): six affine heads, no hidden layer (Sec. 5.2)."""
    W = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], float)
    return Net([3, 6], [(1, 0, W)], [np.full(6, -0.5)])


# ---------------------------------------------------------------------------
# Seeded random nets.
# ---------------------------------------------------------------------------

def sliver_net(h: float = 2.0 ** -28) -> Net:
    """F = z - 1/2 cut by six hidden planes that leave the hidden units
    without effect on F (zero output weights), so every face lies in the plane
    z = 1/2 and the faces tile the square [-1,1]^2 x {1/2} (total area 4).

    Units: x > 3/4, y > 3/4, x + y > 3/2 + h, x > -3/4, y > -3/4,
    -x - y > 3/2.  With h = 2^-28 the first three bound a right triangle with
    legs h at (3/4, 3/4): a face of area h^2/2 = 2^-57 about 1 away from the
    plane's foot point (0, 0, 1/2).  The last three meet in one point
    (-3/4, -3/4): the cell with units 3, 4 and 5 on touches the plane there
    and has a face of zero area.  Every weight and bias is dyadic.
    """
    W1 = np.array([[1, 0, 0], [0, 1, 0], [1, 1, 0], [1, 0, 0], [0, 1, 0], [-1, -1, 0]], np.float64)
    b1 = np.array([-0.75, -0.75, -1.5 - h, 0.75, 0.75, -1.5])
    return Net([3, 6, 1], [(1, 0, W1), (2, 0, np.array([[0.0, 0.0, 1.0]])), (2, 1, np.zeros((1, 6)))],
               [b1, np.array([-0.5])])


def he_mlp(hidden: Sequence[int], seed: int, bias_std: float = 0.01,
           n_in: int = 3, n_out: int = 1) -> Tuple[list, list]:
    """Plain MLP parameters with W ~ N(0, 2/fan_in), b ~ N(0, bias_std^2).

    Draw order W1, b1, W2, b2, ..., W_out, b_out from numpy's PCG64 stream.
    """
    rng = np.random.default_rng(seed)
    sizes = [n_in] + list(hidden) + [n_out]
    Ws, bs = [], []
    for i in range(len(sizes) - 1):
        fan_in = sizes[i]
        Ws.append(rng.normal(0.0, np.sqrt(2.0 / fan_in), (sizes[i + 1], sizes[i])))
        bs.append(rng.normal(0.0, bias_std, sizes[i + 1]))
    return Ws, bs


def mlp_net(Ws: Sequence[np.ndarray], bs: Sequence[np.ndarray]) -> Net:
    widths = [Ws[0].shape[1]] + [W.shape[0] for W in Ws]
    blocks = [(l + 1, l, W) for l, W in enumerate(Ws)]
    return Net(widths, blocks, list(bs))


def random_mlp(hidden: Sequence[int], seed: int, bias_std: float = 0.1) -> Net:
    Ws, bs = he_mlp(hidden, seed, bias_std)
    return mlp_net(Ws, bs)


def c1_net(seed: int = 0) -> Net:
    """F(x) = 0.1 MLP(x) + (max(|x|,|y|,|z|) - 0.5), MLP 3->64->64->1.

    MLP weights W ~ N(0, 2/fan_in), b ~ N(0, 0.01^2), seed 0, draw order
    W1, b1, W2, b2, W3, b3.  The max-norm units are stacked after the MLP
    units of layers 1 and 2 and as the only unit of layer 3, so N = 67+65+1.
    """
    (W1, W2, W3), (b1, b2, b3) = he_mlp([64, 64], seed, 0.01)
    widths = [3, 67, 65, 1, 1]
    B10 = np.zeros((67, 3)); B10[:64] = W1; B10[64:] = np.eye(3)
    B21 = np.zeros((65, 67)); B21[:64, :64] = W2; B21[64, 64:67] = [-2.0, 2.0, 0.0]
    B20 = np.zeros((65, 3)); B20[64] = [1.0, -1.0, 0.0]
    B31 = np.zeros((1, 67)); B31[0, 64:67] = [-2.0, 0.0, 2.0]
    B30 = np.array([[1.0, 0.0, -1.0]])
    B32 = np.zeros((1, 65)); B32[0, 64] = -1.0
    B42 = np.zeros((1, 65)); B42[0, :64] = 0.1 * W3[0]; B42[0, 64] = 1.0
    B41 = np.zeros((1, 67)); B41[0, 64] = 2.0
    B40 = np.array([[-1.0, 0.0, 0.0]])
    B43 = np.array([[1.0]])
    bias = [np.concatenate([b1, np.zeros(3)]), np.concatenate([b2, np.zeros(1)]),
            np.zeros(1), np.array([0.1 * b3[0] - 0.5])]
    blocks = [(1, 0, B10), (2, 1, B21), (2, 0, B20), (3, 1, B31), (3, 0, B30), (3, 2, B32),
              (4, 2, B42), (4, 1, B41), (4, 0, B40), (4, 3, B43)]
    return Net(widths, blocks, bias)


def shortcut_cube_mlp(hidden: Sequence[int], seed: int, scale: float = 0.3) -> Net:
    """``scale * MLP(x) + cube(x)``: a small random net with exact shortcuts.

    Used for brute-force cross-checks: the cube units give a closed surface,
    the random units bend it.  Hidden layers of the MLP are stacked with the
    cube units exactly as in :func:`c1_net` (needs >= 2 MLP hidden layers).
    """
    if len(hidden) != 2:
        raise ValueError("shortcut_cube_mlp takes two MLP hidden layers")
    (W1, W2, W3), (b1, b2, b3) = he_mlp(hidden, seed, 0.05)
    h1, h2 = hidden
    widths = [3, h1 + 3, h2 + 1, 1, 1]
    B10 = np.zeros((h1 + 3, 3)); B10[:h1] = W1; B10[h1:] = np.eye(3)
    B21 = np.zeros((h2 + 1, h1 + 3)); B21[:h2, :h1] = W2; B21[h2, h1:h1 + 3] = [-2.0, 2.0, 0.0]
    B20 = np.zeros((h2 + 1, 3)); B20[h2] = [1.0, -1.0, 0.0]
    B31 = np.zeros((1, h1 + 3)); B31[0, h1:h1 + 3] = [-2.0, 0.0, 2.0]
    B30 = np.array([[1.0, 0.0, -1.0]])
    B32 = np.zeros((1, h2 + 1)); B32[0, h2] = -1.0
    B42 = np.zeros((1, h2 + 1)); B42[0, :h2] = scale * W3[0]; B42[0, h2] = 1.0
    B41 = np.zeros((1, h1 + 3)); B41[0, h1] = 2.0
    B40 = np.array([[-1.0, 0.0, 0.0]])
    B43 = np.array([[1.0]])
    bias = [np.concatenate([b1, np.zeros(3)]), np.concatenate([b2, np.zeros(1)]),
            np.zeros(1), np.array([scale * b3[0] - 0.5])]
    blocks = [(1, 0, B10), (2, 1, B21), (2, 0, B20), (3, 1, B31), (3, 0, B30), (3, 2, B32),
              (4, 2, B42), (4, 1, B41), (4, 0, B40), (4, 3, B43)]
    return Net(widths, blocks, bias)


def random_sphere_like(hidden: Sequence[int], seed: int, radius: float = 0.6,
                       scale: float = 0.5) -> Net:
    """``scale * MLP(x) + (|x|_1 - radius)``: random net with a closed zero set.

    The L1 norm uses |t| = 2 relu(t) - t through three extra units of layer 1
    and an input shortcut to the head.
    """
    Ws, bs = he_mlp(hidden, seed, 0.05)
    L = len(hidden)
    widths = [3, hidden[0] + 3] + list(hidden[1:]) + [1]
    B10 = np.zeros((hidden[0] + 3, 3)); B10[:hidden[0]] = Ws[0]; B10[hidden[0]:] = np.eye(3)
    blocks = [(1, 0, B10)]
    bias = [np.concatenate([bs[0], np.zeros(3)])]
    for l in range(1, L):
        W = np.zeros((hidden[l], widths[l])); W[:, :hidden[l - 1]] = Ws[l]
        blocks.append((l + 1, l, W)); bias.append(bs[l])
    Wout = np.zeros((1, widths[L])); Wout[0, :hidden[L - 1]] = scale * Ws[L][0]
    if L == 1:
        Wout[0, hidden[0]:] = 2.0
        blocks.append((L + 1, L, Wout))
    else:
        blocks.append((L + 1, L, Wout))
        Wl1 = np.zeros((1, widths[1])); Wl1[0, hidden[0]:] = 2.0
        blocks.append((L + 1, 1, Wl1))
    blocks.append((L + 1, 0, -np.ones((1, 3))))
    bias.append(np.array([scale * bs[L][0] - radius]))
    return Net(widths, blocks, bias)


def maxpool_of(nets: Sequence[Net]) -> Net:
    """Union by a final max over single-head sub-networks (Sec. 5.2).

    The sub-networks' hidden layers are placed one after another (sub-net 0's
    layers first), so their codes concatenate; head i reads sub-net i.
    """
    widths = [3]
    blocks = []
    bias = []
    layer_of = []        # per sub-net: map of its layer index -> global layer index
    for net in nets:
        if net.n_heads != 1:
            raise ValueError("sub-networks must have one head")
        base = len(widths) - 1
        m = {0: 0}
        for l in range(1, len(net.widths) - 1):
            m[l] = base + l
            widths.append(net.widths[l])
            bias.append(net.bias[l - 1])
        layer_of.append(m)
    head_layer = len(widths)
    widths.append(len(nets))
    hb = np.zeros(len(nets))
    head_blocks = {}
    for i, net in enumerate(nets):
        m = layer_of[i]
        Lsub = len(net.widths) - 2
        for d, s, W in net.blocks:
            if d <= Lsub:
                blocks.append((m[d], m[s], W))
            else:
                src = m[s]
                Wh = head_blocks.setdefault(src, np.zeros((len(nets), widths[src])))
                Wh[i] += W[0]
        hb[i] = net.bias[-1][0]
    for src, Wh in head_blocks.items():
        blocks.append((head_layer, src, Wh))
    bias.append(hb)
    return Net(widths, blocks, bias)


# ---------------------------------------------------------------------------
# Fitted fixtures (frozen files; produced by am_workloads/fit.py).
# ---------------------------------------------------------------------------

FITTED = {
    # name: (file, sha256 of the file)  -- filled in by fit.py's --record
}


def load_fitted(name: str) -> Net:
    path = os.path.join(DATA_DIR, f"{name}.npz")
    if not os.path.exists(path):
        raise FileNotFoundError(f"fitted fixture {path} missing; run python -m am_workloads.fit {name}")
    return Net.load(path)


# ---------------------------------------------------------------------------
# Shapes sharing one network's weights (latent-conditioned decoders).
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class ShapeBatch:
    """S shapes that share ``net``'s weights; row s of ``shape_bias`` holds the
    biases of every layer >= 1 (layers in order) for shape s."""
    net: Net
    shape_bias: np.ndarray      # [S, sum(widths[1:])]

    @property
    def n_shapes(self) -> int:
        return int(self.shape_bias.shape[0])

    def shape_net(self, s: int) -> Net:
        """The single network that shape s is."""
        row = self.shape_bias[s]
        bias, o = [], 0
        for w in self.net.widths[1:]:
            bias.append(row[o:o + w].copy())
            o += w
        return Net(list(self.net.widths), [(d, k, W.copy()) for d, k, W in self.net.blocks], bias)


def latent_sphere_batch(hidden: Sequence[int], reinject: int, latent_dim: int, n_shapes: int, seed: int,
                        latent_std: float = 0.3, radius=(0.4, 0.8), scale: float = 0.4,
                        log_radii: bool = False) -> ShapeBatch:
    """A latent-conditioned decoder ``scale * MLP([x; z]) + |x|_1 - r_s``.

    The MLP takes [x; z] at layer 1 and again at layer ``reinject`` (a linear
    shortcut from the input, Sec. 5.1); the latent terms W_z z_s are folded
    into the biases of those layers.  Shape s has latent z_s ~ N(0, latent_std^2)
    and radius r_s spread over ``radius``, evenly or (log_radii) geometrically,
    so the shapes' sizes, and cell counts, differ.  The L1 norm uses |t| = 2 relu(t) - t (three extra units
    of layer 1 and an input shortcut to the head).
    """
    rng = np.random.default_rng(seed)
    L = len(hidden)
    if not (2 <= reinject <= L):
        raise ValueError("reinject must name a hidden layer after the first")
    n_in = 3 + latent_dim
    Wx, Wz, bs = [], [], []
    for l in range(L):
        fan = n_in if l == 0 else hidden[l - 1] + (n_in if l + 1 == reinject else 0)
        W = rng.normal(0.0, np.sqrt(2.0 / fan), (hidden[l], fan))
        bs.append(rng.normal(0.0, 0.05, hidden[l]))
        if l == 0:
            Wx.append(W[:, :3]); Wz.append(W[:, 3:])
        elif l + 1 == reinject:
            Wx.append(W); Wz.append(None)
        else:
            Wx.append(W); Wz.append(None)
    Wout = rng.normal(0.0, np.sqrt(2.0 / hidden[-1]), (1, hidden[-1]))
    bout = rng.normal(0.0, 0.05, 1)
    Z = rng.normal(0.0, latent_std, (n_shapes, latent_dim))
    radii = (np.geomspace if log_radii else np.linspace)(radius[0], radius[1], n_shapes)

    widths = [3, hidden[0] + 3] + list(hidden[1:]) + [1]
    B10 = np.zeros((hidden[0] + 3, 3)); B10[:hidden[0]] = Wx[0]; B10[hidden[0]:] = np.eye(3)
    blocks = [(1, 0, B10)]
    for l in range(1, L):
        W = Wx[l]
        if l + 1 == reinject:
            Wh = W[:, :hidden[l - 1]]                  # from the previous layer
            Wxr = W[:, hidden[l - 1]:hidden[l - 1] + 3]  # x re-injected
            Wzr = W[:, hidden[l - 1] + 3:]               # z re-injected (folded into the bias)
            Wz[l] = Wzr
            blocks.append((l + 1, 0, Wxr))
        else:
            Wh = W
        Bp = np.zeros((hidden[l], widths[l])); Bp[:, :hidden[l - 1]] = Wh
        blocks.append((l + 1, l, Bp))
    Bo = np.zeros((1, widths[L])); Bo[0, :hidden[L - 1]] = scale * Wout[0]
    if L == 1:
        Bo[0, hidden[0]:] = 2.0
        blocks.append((L + 1, L, Bo))
    else:
        blocks.append((L + 1, L, Bo))
        B1h = np.zeros((1, widths[1])); B1h[0, hidden[0]:] = 2.0
        blocks.append((L + 1, 1, B1h))
    blocks.append((L + 1, 0, -np.ones((1, 3))))

    rows = []
    for s in range(n_shapes):
        bias = []
        for l in range(L):
            b = bs[l].copy()
            if Wz[l] is not None:
                b = b + Wz[l] @ Z[s]
            if l == 0:
                b = np.concatenate([b, np.zeros(3)])
            bias.append(b)
        bias.append(np.array([scale * bout[0] - radii[s]]))
        rows.append(np.concatenate(bias))
    shape_bias = np.asarray(rows)
    base = [shape_bias[0][o:o + w] for o, w in zip(np.cumsum([0] + widths[1:-1]), widths[1:])]
    return ShapeBatch(Net(widths, blocks, base), shape_bias)


def c4_batch(n_shapes: int = 64) -> ShapeBatch:
    """The batched workload: 64 shapes of one trained latent-conditioned
    decoder, each in its own domain box.

    The decoder (frozen fixture am_workloads/data/c4.npz, written by
    ``python -m am_workloads.fit c4``) is a [x; z] (3 + 256) -> [512] x 8 -> 1
    ReLU MLP with [x; z] entering layer 1 and again layer 4 (fan-in
    512 + 259), trained as an auto-decoder on 64 sphere unions (1-8 spheres
    each, scaled by a log-uniform factor in [0.03, 0.6], ordered by it), one
    latent per shape.  Each latent's terms fold into the biases of layers 1
    and 4 (per-shape bias rows); x re-enters layer 4 as a linear shortcut from
    the input (Sec. 5.1).

    Shape s is marched in the box of half-size h_s centred on a point p_s of
    its surface (c4_boxes.npz; h_s log-spaced from 1.2e-3 to 0.125).  The
    network of shape s takes box coordinates y in [-1, 1]^3, x = p_s + h_s y:
    since relu(t / h) = relu(t) / h for h > 0, every pre-activation of the
    decoder at x equals h_s times that of a network with the decoder's
    weights and biases (b + W_x p_s + W_z z_s) / h_s.  Weights stay shared, the
    codes and the zero set are the decoder's, and faces come out in y.
    """
    z = np.load(os.path.join(DATA_DIR, "c4.npz"), allow_pickle=False)
    box = np.load(os.path.join(DATA_DIR, "c4_boxes.npz"), allow_pickle=False)
    Z = z["Z"].astype(np.float64)[:n_shapes]
    reinject = int(z["reinject"])
    n_w = len([k for k in z.files if k.startswith("W")])
    Ws = [z[f"W{l}"].astype(np.float64) for l in range(n_w)]
    bs = [z[f"b{l}"].astype(np.float64) for l in range(n_w)]
    hidden = [W.shape[0] for W in Ws[:-1]]
    L = len(hidden)
    widths = [3] + hidden + [1]
    blocks = [(1, 0, Ws[0][:, :3])]
    zfold = {1: Ws[0][:, 3:]}
    xfold = {1: Ws[0][:, :3]}
    for l in range(1, L):
        W = Ws[l]
        if l + 1 == reinject:
            h = hidden[l - 1]
            blocks.append((l + 1, l, W[:, :h]))
            blocks.append((l + 1, 0, W[:, h:h + 3]))
            zfold[l + 1] = W[:, h + 3:]
            xfold[l + 1] = W[:, h:h + 3]
        else:
            blocks.append((l + 1, l, W))
    blocks.append((L + 1, L, Ws[-1]))
    rows = []
    for s in range(Z.shape[0]):
        p, hs = box["centre"][s], float(box["half"][s])
        bias = []
        for l in range(1, L + 2):
            b = bs[l - 1].copy()
            if l in zfold:
                b = b + zfold[l] @ Z[s] + xfold[l] @ p
            bias.append(b / hs)
        rows.append(np.concatenate(bias))
    shape_bias = np.asarray(rows)
    base = [shape_bias[0][o:o + w] for o, w in zip(np.cumsum([0] + widths[1:-1]), widths[1:])]
    return ShapeBatch(Net(widths, blocks, base), shape_bias)


def c4_seed_rays(n_shapes: int = 64):
    """Seed rays of the batched workload, one per shape in its box
    coordinates: the segment t e_x, t in [-a_s, a_s], through the surface
    point at the box centre (its ends have opposite signs).  Returns origins,
    directions (o + t d, t in [0, 1]) and shape ids."""
    box = np.load(os.path.join(DATA_DIR, "c4_boxes.npz"), allow_pickle=False)
    a = box["seed_a"][:n_shapes]
    o = np.zeros((n_shapes, 3))
    d = np.zeros((n_shapes, 3))
    o[:, 0] = -a
    d[:, 0] = 2.0 * a
    return o, d, np.arange(n_shapes, dtype=np.int32)


def c4_untrained_batch(n_shapes: int = 64, radius=(0.008, 0.35)) -> ShapeBatch:
    """An untrained stand-in for the batched workload: 64 shapes of one latent-conditioned decoder.

    [x; z] (3 + 256) -> [512] x 8 -> 1 ReLU MLP with [x; z] entering layer 1
    and again layer 4 (fan-in 512 + 259), He-normal weights, biases
    N(0, 0.05^2), latents z_i ~ N(0, 0.01^2), seed 3; the output is
    0.01 * MLP + |x|_1 - r_i with radii geometrically spaced over `radius`, so
    that per-shape cell counts run from about 1e3 to 1e6 (measured: cells grow
    like r^1.85).  The decoder is untrained; the radius term sets each
    shape's size.
    """
    return latent_sphere_batch([512] * 8, reinject=4, latent_dim=256, n_shapes=n_shapes, seed=3,
                               latent_std=0.01, radius=radius, scale=0.01, log_radii=True)



def shifted(net: Net, c) -> Net:
    """The network x -> net(x - c): every block from the input gives its
    destination layer the extra bias -W c."""
    c = np.asarray(c, np.float64)
    bias = [b.copy() for b in net.bias]
    for d, s, W in net.blocks:
        if s == 0:
            bias[d - 1] = bias[d - 1] - W @ c
    return Net(list(net.widths), [(d, s, W.copy()) for d, s, W in net.blocks], bias)


def negated_head(net: Net) -> Net:
    """The network -net(x) (single head): head blocks and bias change sign."""
    L = len(net.widths) - 1
    blocks = [(d, s, -W if d == L else W.copy()) for d, s, W in net.blocks]
    bias = [b.copy() for b in net.bias]
    bias[-1] = -bias[-1]
    return Net(list(net.widths), blocks, bias)


def ensemble_net(n_sub: int = 4, depth: int = 4, width: int = 32, seed: int = 5) -> Net:
    """A max-pooled ensemble in the form of the paper's local decoders (Sec. 5.2,
    Table 7: 4 sub-networks of depth 4 and width 32 joined by a max).

    Sub-network i is an occupancy-style logit, positive inside:
    r_i - |x - c_i|_1 - 0.3 MLP_i(x - c_i), with MLP_i a He-normal ReLU MLP of
    `depth` hidden layers of `width` units (seed + i), centre c_i ~ U[-0.35, 0.35]^3
    and radius r_i ~ U[0.25, 0.45] (drawn in that order from seed); the max of
    the logits is positive on the union of the insides.  Untrained: a synthetic
    stand-in for the paper's trained decoders.
    """
    subs = []
    for i, (c, r) in enumerate(ensemble_centres(n_sub, seed)):
        sub = random_sphere_like([width] * depth, seed=seed + i, radius=r, scale=0.3)
        subs.append(negated_head(shifted(sub, c)))
    return maxpool_of(subs)


def ensemble_centres(n_sub: int = 4, seed: int = 5):
    """(centre, radius) of each sub-network of ensemble_net (same draws)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_sub):
        c = rng.uniform(-0.35, 0.35, 3)
        r = float(rng.uniform(0.25, 0.45))
        out.append((c, r))
    return out
