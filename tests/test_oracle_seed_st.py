"""Pins of the oracle's sphere-tracing seeding (Sec. 4.3.1, Eqn (SphereTracing)).

Closed forms: on the cube net max(|x|,|y|,|z|) - 0.5 and the max-pooled cube
(six heads +-x_i - 0.5) the gradient in a cell is the unit axis of the
largest coordinate, so from a point inside the cube one step moves that
coordinate to +-0.5 and leaves the others; on the octahedron |x|+|y|+|z| - 0.75 the gradient is the sign vector
(|g|^2 = 3), so one step from a point well inside an orthant lands on
x - (|x|_1 - 0.75) sign(x) / 3.  Definition: on other nets every settled
point has F = 0 (plain forward pass) and the forward-pass code there is the
returned code.
"""
import numpy as np
import pytest

from am_workloads import nets
from oracle import brute
from oracle import oracle as O


def _cube_points(n, seed):
    rng = np.random.default_rng(seed)
    pts = []
    while len(pts) < n:
        x = rng.uniform(-0.45, 0.45, 3)            # inside: the largest coordinate stays largest
        a = np.sort(np.abs(x))
        if a[2] - a[1] > 1e-3 and a[0] > 1e-3:        # clear of ties and planes
            pts.append(x)
    return np.array(pts)


def cube_pin(lib_path=None, net_fn=nets.cube_net):
    on = O.OracleNet(net_fn(), lib_path) if lib_path else O.OracleNet(net_fn())
    for x0 in _cube_points(40, 1):
        st, x, code, am, it = on.seed_st(x0)
        k = int(np.argmax(np.abs(x0)))
        want = x0.copy()
        want[k] = np.sign(x0[k]) * 0.5
        assert st == 0 and it == 1
        assert np.max(np.abs(x - want)) <= 1e-15, (x0, x, want)   # F carries rounding of |y| - |x|


def octahedron_pin(lib_path=None):
    net = nets.octahedron_net()
    on = O.OracleNet(net, lib_path) if lib_path else O.OracleNet(net)
    rng = np.random.default_rng(2)
    n = 0
    while n < 40:
        x0 = rng.uniform(-0.6, 0.6, 3)
        if np.abs(x0).min() < 0.2:
            continue
        n += 1
        st, x, code, am, it = on.seed_st(x0)
        want = x0 - (np.abs(x0).sum() - 0.75) * np.sign(x0) / 3.0
        assert st == 0 and it == 1
        assert np.max(np.abs(x - want)) <= 1e-15


def definition_pin(net, lib_path=None, n=60, seed=3):
    on = O.OracleNet(net, lib_path) if lib_path else O.OracleNet(net)
    rng = np.random.default_rng(seed)
    settled = 0
    for x0 in rng.uniform(-0.8, 0.8, (n, 3)):
        st, x, code, am, it = on.seed_st(x0)
        if st != 0:
            continue
        settled += 1
        F = brute.forward_pre(net, x)[0][net.n_hidden:].max()
        assert abs(F) <= 1e-12
        c2, a2, _ = on.code(x)
        assert np.array_equal(c2, code) and a2 == am
    assert settled >= n // 2


def test_cube_one_step_closed_form():
    cube_pin()


def test_maxpool_cube_one_step_closed_form():
    cube_pin(net_fn=nets.maxpool_cube_net)


def test_octahedron_one_step_closed_form():
    octahedron_pin()


@pytest.mark.parametrize("name", ["c1", "sphere_like", "maxpool"])
def test_settled_points_are_surface_points_of_their_cell(name):
    net = {"c1": nets.c1_net,
           "sphere_like": lambda: nets.random_sphere_like([24, 24], seed=5, radius=0.6, scale=0.4),
           "maxpool": lambda: nets.maxpool_of([nets.random_sphere_like([8], seed=7, radius=0.5, scale=0.3),
                                               nets.random_sphere_like([6], seed=8, radius=0.4, scale=0.3)])}[name]()
    definition_pin(net)


def test_zero_gradient_and_outside_box_are_reported():
    # a constant net (zero weights) has no gradient anywhere
    w = [3, 2, 1]
    blocks = [(1, 0, np.zeros((2, 3))), (2, 1, np.zeros((1, 2)))]
    net = nets.Net(w, blocks, [np.array([0.1, 0.1]), np.array([0.5])])
    st, *_ = O.OracleNet(net).seed_st(np.zeros(3))
    assert st == 2
    # x - 2 = 0 only at x = 2, outside the box
    blocks = [(1, 0, np.zeros((1, 3))), (2, 0, np.array([[1.0, 0.0, 0.0]]))]
    net = nets.Net([3, 1, 1], blocks, [np.zeros(1), np.array([-2.0])])
    st, x, *_ = O.OracleNet(net).seed_st(np.zeros(3))
    assert st == 3 and abs(x[0] - 2.0) < 1e-15
