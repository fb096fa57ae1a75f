"""The oracle's pins catch plausible mistakes.

Each mutant is the oracle compiled with one planted mistake (ORC_MUTATE=k in
oracle/am_oracle.c): a dropped bias, a flipped constraint orientation, a
missing ReLU mask, dropped shortcut blocks, a reversed max-pool comparison, a
wrong edge pair in the vertex solve, the wrong tie rule, a wrong neighbour
flip, a transposed weight block, ON vertices treated as outside, two
sphere-tracing seeding mistakes (no gradient normalisation, wrong head) and
two pivoting mistakes (no positive-length-edge rule, no orientation fix) and
the area taken by the absolute shoelace instead of from the first vertex.  The
test runs a battery of the pins (closed-form nets, brute force, Lemma 1,
closedness) against every mutant and asserts that at least one pin fails.
"""
import os

import numpy as np
import pytest

import meshcheck as MC
import test_oracle_pivot as PV
import test_oracle_seed_st as ST
from am_workloads import nets
from oracle import brute
from oracle import oracle as O

MUTANTS = {
    1: "bias dropped from the chain",
    2: "constraint orientation flipped",
    3: "ReLU mask ignored in the chain",
    4: "shortcut blocks dropped",
    5: "max-pool comparison reversed",
    6: "vertex solved from the wrong edge pair",
    7: "state tie rule a>=0 -> on",
    8: "neighbour flips the wrong unit",
    9: "square weight blocks transposed",
    10: "ON vertices treated as outside",
    11: "sphere-tracing step not divided by |grad F|^2",
    12: "sphere-tracing gradient taken from head 0, not the argmax head",
    13: "pivoting accepts a plane without a positive-length edge on it",
    14: "pivoting keeps the walk's orientation",
    15: "face area by the absolute shoelace about the frame origin",
}


def _net_mlp_square():
    net = nets.random_mlp([5, 5], seed=77, bias_std=0.3)
    X = np.random.default_rng(0).uniform(-1, 1, (4096, 3))
    shift = float(np.mean(brute.forward_pre(net, X)[:, -1])) + 0.0123
    bias = [b.copy() for b in net.bias]
    bias[-1] = bias[-1] - shift
    return nets.Net(net.widths, net.blocks, bias)


def _net_maxpool():
    subs = []
    for s, h in ((1, [4]), (2, [3])):
        net = nets.random_mlp(h, seed=600 + s, bias_std=0.3)
        X = np.random.default_rng(s).uniform(-1, 1, (4096, 3))
        shift = float(np.mean(brute.forward_pre(net, X)[:, -1])) + 0.0123
        bias = [b.copy() for b in net.bias]
        bias[-1] = bias[-1] - shift
        subs.append(nets.Net(net.widths, net.blocks, bias))
    return nets.maxpool_of(subs)


def _pin_exact(lib_path, net, F, V, area, vol):
    on = O.OracleNet(net, lib_path)
    st, x, code, am = on.seed_ray(np.zeros(3), np.array([0.9, 0.13, 0.07]))
    assert st == 0
    mesh = on.march(code[None], np.array([am]))
    assert mesh.n_faces == F
    chi, v, e, f = MC.euler(mesh, net.n_hidden)
    assert chi == 2 and v == V
    A, Vol = MC.area_volume(mesh)
    assert abs(A - area) < 1e-12 and abs(Vol - vol) < 1e-12


def _pin_sliver(lib_path):
    """The sliver net: 14 faces tiling the square (area 4), one of area 2^-57."""
    net = nets.sliver_net()
    on = O.OracleNet(net, lib_path)
    code, am, _ = on.code(np.array([0.0, 0.0, 0.5]))
    mesh = on.march(code[None], np.array([am]))
    assert mesh.n_faces == 14
    A, _ = MC.area_volume(mesh)
    assert abs(A - 4.0) < 1e-12
    _, _, area, _ = on.face(np.array([0b011011], np.uint64))
    assert area == 2.0 ** -57


def _pin_brute(lib_path, net):
    ref = brute.all_faces(net)
    on = O.OracleNet(net, lib_path)
    keys = list(ref)
    codes = np.array([brute.bits_to_words(k[0], on.W) for k in keys], np.uint64).reshape(-1, on.W)
    mesh = on.march(codes, np.array([k[1] for k in keys], np.int32))
    got = {(brute.words_to_bits(mesh.codes[f], net.n_hidden), int(mesh.argmax[f])): mesh.face(f)
           for f in range(mesh.n_faces)}
    assert set(got) == set(ref)
    for k, (ids, vs) in ref.items():
        assert np.array_equal(got[k][0], ids)
        assert np.max(np.abs(got[k][1] - vs)) <= 1e-9
    bad, _ = MC.edge_pairing(mesh, n_hidden=net.n_hidden)
    assert bad == 0


def _pin_lemma1(lib_path, net):
    on = O.OracleNet(net, lib_path)
    rng = np.random.default_rng(5)
    for x in rng.uniform(-0.9, 0.9, (40, 3)):
        code, am, F = on.code(x)
        rows = on.chain(code)
        assert np.allclose(rows @ np.append(x, 1.0), brute.forward_pre(net, x)[0], atol=1e-12)


def _pin_tie(lib_path):
    on = O.OracleNet(nets.cube_net(), lib_path)
    code, am, F = on.code(np.zeros(3))
    assert int(code[0]) == 0


def _pin_c1_closed(lib_path):
    net = nets.c1_net()
    on = O.OracleNet(net, lib_path)
    st, x, code, am = on.seed_ray(np.zeros(3), np.array([1.0, 0.0, 0.0]))
    assert st == 0
    mesh = on.march(code[None], np.array([am]), max_cells=200000)
    bad, dom = MC.edge_pairing(mesh, n_hidden=net.n_hidden)
    assert bad == 0 and dom == 0
    assert MC.euler(mesh, net.n_hidden)[0] == 2


def _battery(lib_path):
    """Runs every pin; returns the names of those that failed."""
    pins = [
        ("cube", lambda: _pin_exact(lib_path, nets.cube_net(), 32, 26, 6.0, 1.0)),
        ("maxpool_cube", lambda: _pin_exact(lib_path, nets.maxpool_cube_net(), 6, 8, 6.0, 1.0)),
        ("octahedron_split", lambda: _pin_exact(lib_path, nets.octahedron_split_net(), 12, 8,
                                                4.0 * 3 ** 0.5 * 0.5625, 0.5625)),
        ("tie", lambda: _pin_tie(lib_path)),
        ("lemma1_c1", lambda: _pin_lemma1(lib_path, nets.c1_net())),
        ("brute_mlp", lambda: _pin_brute(lib_path, _net_mlp_square())),
        ("brute_maxpool", lambda: _pin_brute(lib_path, _net_maxpool())),
        ("brute_cube", lambda: _pin_brute(lib_path, nets.shortcut_cube_mlp([4, 4], 301, 0.3))),
        ("c1_closed", lambda: _pin_c1_closed(lib_path)),
        ("st_cube", lambda: ST.cube_pin(lib_path)),
        ("st_maxpool_cube", lambda: ST.cube_pin(lib_path, nets.maxpool_cube_net)),
        ("st_octahedron", lambda: ST.octahedron_pin(lib_path)),
        ("pivot_cube", lambda: PV.pin_exact(lib_path, nets.cube_net)),
        ("pivot_octahedron_split", lambda: PV.pin_exact(lib_path, nets.octahedron_split_net)),
        ("pivot_brute", lambda: PV.pin_brute(lib_path, _net_mlp_square())),
        ("sliver", lambda: _pin_sliver(lib_path)),
    ]
    failed = []
    for name, fn in pins:
        try:
            fn()
        except Exception:          # an assertion or an error both count as caught
            failed.append(name)
    return failed


def test_unmutated_oracle_passes_battery():
    assert _battery(O.LIB_PATH) == []


@pytest.mark.parametrize("k", sorted(MUTANTS))
def test_mutant_is_caught(k, tmp_path):
    path = os.path.join(str(tmp_path), f"liborc_mut{k}.so")
    O.build(out=path, mutate=k)
    failed = _battery(path)
    assert failed, f"mutant {k} ({MUTANTS[k]}) passed every pin"
