"""Pins of the RC-estimation oracle (oracle/rc_estimate.py) on the CPU: the
tree's total wire length against scipy's minimum spanning tree of the same
Manhattan distances, closed forms for two-pin and collinear nets, the tree
structure, and the Elmore delay of an estimated single wire through the
timing oracle."""
import numpy as np
import pytest
from scipy.sparse.csgraph import minimum_spanning_tree

import oracle
from oracle import rc_estimate as R
from paper_2511_11660_amd import synth


def _length(parent, res, cap, rx=1.0):
    """Total wire length of an estimated tree built with unit resistance rx
    along both axes (R = length)."""
    return float(np.sum(res.astype(np.float64))) / rx


@pytest.mark.parametrize("seed", range(8))
def test_tree_length_is_the_minimum_spanning_tree(seed):
    rng = np.random.default_rng(seed)
    for k in (1, 2, 3, 7, 20, 45):
        px = rng.uniform(0, 100, k + 1).astype(np.float32)
        py = rng.uniform(0, 100, k + 1).astype(np.float32)
        parent, res, cap, node_of = R.estimate_net(px, py, 1.0, 1.0, 0.0, 0.0)
        dm = np.abs(px[:, None].astype(np.float64) - px[None, :]) + np.abs(py[:, None].astype(np.float64) - py[None, :])
        mst = minimum_spanning_tree(dm).toarray().sum()
        assert _length(parent, res, cap) == pytest.approx(mst, rel=1e-6)


def test_two_pin_net_closed_form():
    rx, ry, cx, cy = 0.003, 0.002, 0.25, 0.15
    parent, res, cap, node_of = R.estimate_net([10.0, 40.0], [5.0, -15.0], rx, ry, cx, cy)
    assert list(parent) == [-1, 0, 1]
    assert node_of.tolist() == [0, 2]
    np.testing.assert_allclose(res, [0.0, rx * 30.0, ry * 20.0], rtol=1e-6)
    np.testing.assert_allclose(cap, [0.0, cx * 30.0, cy * 20.0], rtol=1e-6)


def test_collinear_pins_form_a_chain_in_x_order():
    rng = np.random.default_rng(3)
    xs = rng.permutation(np.arange(12, dtype=np.float32) * 7.0)
    py = np.full(12, 3.0, np.float32)
    parent, res, cap, node_of = R.estimate_net(xs, py, 1.0, 1.0, 1.0, 1.0)
    assert _length(parent, res, cap) == pytest.approx(float(xs.max() - xs.min()))
    # every pin joins next to a neighbour in x: each tree edge spans one gap of 7
    edges = res[1::2]
    np.testing.assert_allclose(edges, 7.0)
    assert np.all(res[2::2] == 0.0) and np.all(cap[2::2] == 0.0)


def test_tree_structure_on_a_design():
    d = synth.generate(synth.tiny_config(seed=5))
    x, y = synth.place(d, seed=2)
    rc = R.estimate_rc(d, x, y, 0.002, 0.002, 0.2, 0.2)
    ptr = rc["net_node_ptr"]
    assert ptr[-1] == d.n_nets + 2 * d.n_sinks
    nsp = np.asarray(d.net_sink_ptr)
    for n in range(d.n_nets):
        a, b = ptr[n], ptr[n + 1]
        par = rc["parent"][a:b]
        assert par[0] == -1 and np.all(par[1:] < np.arange(1, b - a)) and np.all(par[1:] >= 0)
        sn = rc["sink_node"][nsp[n]:nsp[n + 1]]
        assert sorted(sn.tolist()) == list(range(2, b - a, 2))  # every pin node once
    assert np.all(rc["res_kohm"] >= 0) and np.all(rc["cap_ff"] >= 0)


def test_elmore_delay_of_an_estimated_wire():
    """PI -> BUF with the sink 60 um away along x: the estimated tree is one
    x segment (R = r L, C = c L at the corner) then a zero-length y segment
    ending at the sink, so the sink's Elmore delay is r L (c L + Cpin)."""
    from designs import CIN, COUT, PI, PO, make_design, planar_table, single_segment_net
    kinds = [PI, CIN, COUT, PO]
    cells = [(0, [1], 2)]
    nets = [single_segment_net(0, [1], 0.01, 1.0), single_segment_net(2, [3], 0.01, 1.0)]
    t = planar_table(5, 0.1, 1.0)
    tables = np.stack([np.stack([t, t, planar_table(3, 0.05, 2.0), planar_table(3, 0.05, 2.0)])])
    d = make_design(kinds, cells, nets, n_inputs=[1], sense=[0], pin_cap=[1.5], tables=tables, po_rat=500.0)
    r_u, c_u, L = 0.004, 0.3, 60.0
    x = np.array([0.0, L, L, L + 10.0], np.float32)
    y = np.zeros(4, np.float32)
    rc = R.estimate_rc(d, x, y, r_u, r_u, c_u, c_u)
    e = synth.with_rc(d, rc)
    o = oracle.sta(e)
    assert o["d_sink"][0] == pytest.approx(r_u * L * (c_u * L + 1.5), rel=1e-6)


def test_position_gradient_is_the_derivative_of_a_linear_objective():
    """J = sum of fixed weights times every node's R and C: the position
    gradient against central differences of the estimator itself, with the
    tree fixed (a perturbation that changes the pin's net's tree is skipped;
    only that net's terms change, so only it is re-estimated).  Positions are
    multiples of 1/8 um and the unit values powers of two, so every R and C
    is exact in FP32 and a step of 1/64 um is exact too."""
    d = synth.generate(synth.tiny_config(seed=6))
    rng = np.random.default_rng(5)
    x = (rng.integers(0, 800, d.n_pins) / 8.0).astype(np.float32)
    y = (rng.integers(0, 800, d.n_pins) / 8.0).astype(np.float32)
    w = (2.0 ** -9, 2.0 ** -8, 2.0 ** -3, 2.0 ** -2)
    rc = R.estimate_rc(d, x, y, *w)
    wr = rng.uniform(-1, 1, rc["parent"].size)
    wc = rng.uniform(-1, 1, rc["parent"].size)
    gx, gy = R.estimate_rc_backward(d, x, y, rc, *w, wr, wc)
    nsp = np.asarray(d.net_sink_ptr)
    net_of = np.full(d.n_pins, -1)
    net_of[d.net_driver] = np.arange(d.n_nets)
    net_of[d.net_sink_pin] = np.repeat(np.arange(d.n_nets), np.diff(nsp))
    ptr = rc["net_node_ptr"]
    h = np.float32(1.0 / 64)
    checked = 0
    for p in rng.choice(np.flatnonzero(net_of >= 0), 300, replace=False):
        n = net_of[p]
        pins = np.concatenate([[d.net_driver[n]], d.net_sink_pin[nsp[n]:nsp[n + 1]]])
        a, b = ptr[n], ptr[n + 1]
        for g, axis in ((gx, 0), (gy, 1)):
            js = []
            for sgn in (1, -1):
                xy = [x[pins].copy(), y[pins].copy()]
                xy[axis][pins == p] += sgn * h
                par, res, cap, node_of = R.estimate_net(xy[0], xy[1], *w)
                if not (np.array_equal(par, rc["parent"][a:b])
                        and np.array_equal(node_of[1:], rc["sink_node"][nsp[n]:nsp[n + 1]])):
                    break  # another tree or join order
                js.append(np.dot(wr[a:b], res.astype(np.float64)) + np.dot(wc[a:b], cap.astype(np.float64)))
            if len(js) < 2:
                continue
            fd = (js[0] - js[1]) / (2 * float(h))
            # a zero-length segment has a kink: sgn(0) = 0 takes the average of both sides
            assert g[p] == pytest.approx(fd, rel=1e-9, abs=1e-9), (p, axis, g[p], fd)
            checked += 1
    assert checked > 400


def test_position_gradient_of_a_two_pin_net():
    """One wire from (0, 0) to (L, H): R = r_x L + r_y H, C = c_x L + c_y H;
    dJ/dx of the sink = r_x gR_corner + c_x gC_corner, the driver's the negative."""
    from types import SimpleNamespace
    d = SimpleNamespace(n_pins=2, n_nets=1, n_sinks=1, net_driver=np.array([0]), net_sink_ptr=np.array([0, 1]),
                        net_sink_pin=np.array([1]))
    x = np.array([0.0, 30.0], np.float32)
    y = np.array([0.0, -20.0], np.float32)
    rc = R.estimate_rc(d, x, y, 0.5, 0.25, 2.0, 4.0)
    gR = np.array([9.0, 3.0, 5.0])
    gC = np.array([9.0, 7.0, 11.0])
    gx, gy = R.estimate_rc_backward(d, x, y, rc, 0.5, 0.25, 2.0, 4.0, gR, gC)
    assert gx.tolist() == [-(0.5 * 3 + 2.0 * 7), 0.5 * 3 + 2.0 * 7]
    assert gy.tolist() == [0.25 * 5 + 4.0 * 11, -(0.25 * 5 + 4.0 * 11)]  # the sink is below: sgn = -1
