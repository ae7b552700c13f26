"""Pins of the RC-estimation oracle (oracle/rc_estimate.py) on the CPU.

The tree is the rectilinear shortest-path (Takahashi-Matsuyama) Steiner
heuristic; it is pinned by what holds independently of its relaxation code:
its length never exceeds the rectilinear minimum spanning tree (scipy) nor
falls below the exact rectilinear Steiner minimum tree (Hanan-grid brute
force, Hanan's theorem); every join step checked against distances to the
rasterized wires built so far; the RC tree's geometry (every piece runs
along one axis between points of the wires, the pieces add up to the step
distances); closed forms for two-pin, collinear and T-shaped nets (Elmore
through the timing oracle); and the position gradient against central
differences."""
import itertools

import numpy as np
import pytest
from scipy.sparse.csgraph import minimum_spanning_tree

import oracle
from oracle import rc_estimate as R
from paper_2511_11660_amd import synth


def _length(res, rx=1.0):
    """Total wire length of an estimated tree built with unit resistance rx
    along both axes (R = length)."""
    return float(np.sum(res.astype(np.float64))) / rx


def _mst(px, py):
    """Rectilinear minimum spanning tree length (scipy; coincident points,
    whose zero distance scipy would read as "no edge", are merged first)."""
    pts = sorted({(float(a), float(b)) for a, b in zip(px, py)})
    p = np.array(pts, np.float64)
    dm = np.abs(p[:, None, :] - p[None, :, :]).sum(-1)
    return float(minimum_spanning_tree(dm).toarray().sum())


def _rsmt_exact(px, py):
    """Exact rectilinear Steiner minimum tree length: by Hanan's theorem some
    optimal tree has its Steiner points on the Hanan grid, at most n - 2 of
    them, so the minimum over those point sets of the spanning tree of
    terminals plus points is the optimum."""
    n = len(px)
    term = {(float(a), float(b)) for a, b in zip(px, py)}
    hanan = [(a, b) for a in sorted(set(map(float, px))) for b in sorted(set(map(float, py))) if (a, b) not in term]
    best = _mst(px, py)
    for m in range(1, n - 1):
        for extra in itertools.combinations(hanan, m):
            xs = list(map(float, px)) + [e[0] for e in extra]
            ys = list(map(float, py)) + [e[1] for e in extra]
            best = min(best, _mst(xs, ys))
    return best


@pytest.mark.parametrize("seed", range(6))
def test_length_between_exact_steiner_and_spanning_tree(seed):
    rng = np.random.default_rng(seed)
    for trial in range(30):
        k = int(rng.integers(1, 5))  # up to 5 pins: the exact optimum by brute force
        px = rng.integers(0, 12, k + 1).astype(np.float32) * 2.5
        py = rng.integers(0, 12, k + 1).astype(np.float32) * 2.5
        parent, res, cap, node_of = R.estimate_net(px, py, 1.0, 1.0, 0.0, 0.0)
        L = _length(res)
        assert _rsmt_exact(px, py) <= L + 1e-9 <= _mst(px, py) + 2e-9, (px, py)


@pytest.mark.parametrize("seed", range(4))
def test_never_longer_than_the_spanning_tree_and_shorter_on_average(seed):
    rng = np.random.default_rng(100 + seed)
    ratios = []
    for k in (1, 2, 3, 7, 20, 45, 120):
        px = rng.uniform(0, 100, k + 1).astype(np.float32)
        py = rng.uniform(0, 100, k + 1).astype(np.float32)
        parent, res, cap, node_of = R.estimate_net(px, py, 1.0, 1.0, 0.0, 0.0)
        mst = _mst(px, py)
        assert _length(res) <= mst * (1 + 1e-6)
        if k >= 7:
            ratios.append(_length(res) / mst)
    assert np.mean(ratios) < 0.97  # Steiner points pay off on nets of several pins


def _raster(a, b):
    """Integer points of the axis-parallel segment from a to b."""
    (ax, ay), (bx, by) = a, b
    if ax == bx:
        return {(ax, y) for y in range(min(ay, by), max(ay, by) + 1)}
    assert ay == by
    return {(x, ay) for x in range(min(ax, bx), max(ax, bx) + 1)}


@pytest.mark.parametrize("seed", range(5))
def test_join_steps_against_rasterized_wires(seed):
    """Integer coordinates: the wires built so far are rasterized point by
    point; at every step the joining pin is the remaining pin nearest to them
    (lowest index among ties), at that distance, from a point of them that
    lies on the recorded segment."""
    rng = np.random.default_rng(seed)
    for trial in range(25):
        k = int(rng.integers(1, 11))
        px = rng.integers(0, 16, k + 1)
        py = rng.integers(0, 16, k + 1)
        steps = R.sph_net(px.astype(np.float32), py.astype(np.float32))
        wires = {(int(px[0]), int(py[0]))}
        segs = {0: wires.copy()}
        left = set(range(1, k + 1))
        for t, st in enumerate(steps, 1):
            d = {u: min(abs(int(px[u]) - a) + abs(int(py[u]) - b) for a, b in wires) for u in left}
            dmin = min(d.values())
            j = st["j"]
            assert j == min(u for u in left if d[u] == dmin), (t, d, j)
            q = (int(st["q"][0]), int(st["q"][1]))
            assert q in segs[st["sigma"]]
            assert abs(int(px[j]) - q[0]) + abs(int(py[j]) - q[1]) == dmin
            corner = (int(px[j]), q[1])
            segs[2 * t - 1] = _raster(q, corner)
            segs[2 * t] = _raster(corner, (int(px[j]), int(py[j])))
            wires |= segs[2 * t - 1] | segs[2 * t]
            left.remove(j)


@pytest.mark.parametrize("seed", range(5))
def test_rc_tree_geometry(seed):
    """Every node sits at a point of the wires: each piece runs along its
    axis only (the other coordinate equal to its parent's), its R is the
    coordinate difference, each pin's node is at the pin, parents precede
    children, and the pieces add up to the join distances."""
    rng = np.random.default_rng(20 + seed)
    for trial in range(20):
        k = int(rng.integers(1, 30))
        px = rng.integers(0, 40, k + 1).astype(np.float32)
        py = rng.integers(0, 40, k + 1).astype(np.float32)
        parent, res, cap, node_of, src, ax = R.build_net(px, py, 1.0, 1.0, 1.0, 1.0)
        m = 3 * k + 1
        assert parent.size == m and parent[0] == -1
        assert np.all(parent[1:] < np.arange(1, m)) and np.all(parent[1:] >= 0)
        nx, ny = px[src[:, 0]], py[src[:, 1]]
        for i in range(1, m):
            w = parent[i]
            if ax[i] == 0:
                assert ny[i] == ny[w] and res[i] == abs(nx[i] - nx[w])
            else:
                assert nx[i] == nx[w] and res[i] == abs(ny[i] - ny[w])
        assert np.array_equal(nx[node_of], px) and np.array_equal(ny[node_of], py)
        assert sorted(node_of.tolist()) == sorted(set(node_of.tolist()))
        steps = R.sph_net(px, py)
        joined = sum(abs(float(px[s["j"]]) - float(s["q"][0])) + abs(float(py[s["j"]]) - float(s["q"][1]))
                     for s in steps)
        assert _length(res) == joined


def test_two_pin_net_closed_form():
    rx, ry, cx, cy = 0.003, 0.002, 0.25, 0.15
    parent, res, cap, node_of = R.estimate_net([10.0, 40.0], [5.0, -15.0], rx, ry, cx, cy)
    # D, the attach point on the driver (zero piece), the corner, the pin
    assert list(parent) == [-1, 0, 1, 2]
    assert node_of.tolist() == [0, 3]
    np.testing.assert_allclose(res, [0.0, 0.0, rx * 30.0, ry * 20.0], rtol=1e-6)
    np.testing.assert_allclose(cap, [0.0, 0.0, cx * 30.0, cy * 20.0], rtol=1e-6)


def test_collinear_pins_form_one_wire():
    rng = np.random.default_rng(3)
    xs = rng.permutation(np.arange(12, dtype=np.float32) * 7.0)
    py = np.full(12, 3.0, np.float32)
    parent, res, cap, node_of = R.estimate_net(xs, py, 1.0, 1.0, 1.0, 1.0)
    assert _length(res) == pytest.approx(float(xs.max() - xs.min()))
    # no piece crosses a pin: every non-zero piece spans exactly one gap of 7
    nz = res[res > 0]
    np.testing.assert_allclose(nz, 7.0)


def test_t_junction_elmore():
    """Driver at the origin, sink a 10 um along x, sink b at (5, 5): a joins
    first (tie at 10, lower index), b then attaches to the middle of a's wire
    (distance 5), so the tree is a 10 um trunk with a 5 um branch from its
    midpoint: 15 um, the Steiner optimum, where a spanning tree needs 20.
    Elmore delay to b: r 5 (c 15 + Ca + Cb) + r 5 (c 5 + Cb); to a:
    r 5 (c 15 + Ca + Cb) + r 5 (c 5 + Ca)."""
    from designs import CIN, COUT, PI, PO, make_design, planar_table, single_segment_net
    kinds = [PI, CIN, CIN, COUT, COUT, PO, PO]
    cells = [(0, [1], 3), (0, [2], 4)]
    nets = [single_segment_net(0, [1, 2], 0.01, 1.0), single_segment_net(3, [5], 0.01, 1.0),
            single_segment_net(4, [6], 0.01, 1.0)]
    t = planar_table(5, 0.1, 1.0)
    tables = np.stack([np.stack([t, t, planar_table(3, 0.05, 2.0), planar_table(3, 0.05, 2.0)])])
    ca, cb = 1.5, 1.5
    d = make_design(kinds, cells, nets, n_inputs=[1], sense=[0], pin_cap=[ca], tables=tables, po_rat=500.0)
    r_u, c_u = 0.004, 0.25
    x = np.array([0.0, 10.0, 5.0, 10.0, 5.0, 20.0, 20.0], np.float32)
    y = np.array([0.0, 0.0, 5.0, 0.0, 5.0, 0.0, 5.0], np.float32)
    rc = R.estimate_rc(d, x, y, r_u, r_u, c_u, c_u)
    assert _length(rc["res_kohm"][: rc["net_node_ptr"][1]], r_u) == pytest.approx(15.0)
    e = synth.with_rc(d, rc)
    o = oracle.sta(e)
    trunk = r_u * 5 * (c_u * 15 + ca + cb)
    assert o["d_sink"][0] == pytest.approx(trunk + r_u * 5 * (c_u * 5 + ca), rel=1e-6)
    assert o["d_sink"][1] == pytest.approx(trunk + r_u * 5 * (c_u * 5 + cb), rel=1e-6)


def test_tree_structure_on_a_design():
    d = synth.generate(synth.tiny_config(seed=5))
    x, y = synth.place(d, seed=2)
    rc = R.estimate_rc(d, x, y, 0.002, 0.002, 0.2, 0.2)
    ptr = rc["net_node_ptr"]
    assert ptr[-1] == d.n_nets + 3 * d.n_sinks
    nsp = np.asarray(d.net_sink_ptr)
    for n in range(d.n_nets):
        a, b = ptr[n], ptr[n + 1]
        par = rc["parent"][a:b]
        assert par[0] == -1 and np.all(par[1:] < np.arange(1, b - a)) and np.all(par[1:] >= 0)
        sn = rc["sink_node"][nsp[n]:nsp[n + 1]]
        assert len(set(sn.tolist())) == sn.size and np.all(sn > 0) and np.all(sn < b - a)
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
                par, res, cap, node_of, src, ax = R.build_net(xy[0], xy[1], *w)
                ref = R.build_net(x[pins], y[pins], *w)
                if not (np.array_equal(par, rc["parent"][a:b])
                        and np.array_equal(node_of[1:], rc["sink_node"][nsp[n]:nsp[n + 1]])
                        and np.array_equal(src, ref[4])):
                    break  # another tree, join order or clamp choice
                js.append(np.dot(wr[a:b], res.astype(np.float64)) + np.dot(wc[a:b], cap.astype(np.float64)))
            if len(js) < 2:
                continue
            fd = (js[0] - js[1]) / (2 * float(h))
            # a zero-length segment has a kink: sgn(0) = 0 takes the average of both sides
            assert g[p] == pytest.approx(fd, rel=1e-9, abs=1e-9), (p, axis, g[p], fd)
            checked += 1
    assert checked > 300


def test_position_gradient_of_a_two_pin_net():
    """One wire from (0, 0) to (L, H): R = r_x L + r_y H, C = c_x L + c_y H;
    dJ/dx of the sink = r_x gR_corner + c_x gC_corner, the driver's the negative."""
    from types import SimpleNamespace
    d = SimpleNamespace(n_pins=2, n_nets=1, n_sinks=1, net_driver=np.array([0]), net_sink_ptr=np.array([0, 1]),
                        net_sink_pin=np.array([1]))
    x = np.array([0.0, 30.0], np.float32)
    y = np.array([0.0, -20.0], np.float32)
    rc = R.estimate_rc(d, x, y, 0.5, 0.25, 2.0, 4.0)
    gR = np.array([9.0, 13.0, 3.0, 5.0])
    gC = np.array([9.0, 17.0, 7.0, 11.0])
    gx, gy = R.estimate_rc_backward(d, x, y, rc, 0.5, 0.25, 2.0, 4.0, gR, gC)
    assert gx.tolist() == [-(0.5 * 3 + 2.0 * 7), 0.5 * 3 + 2.0 * 7]
    assert gy.tolist() == [0.25 * 5 + 4.0 * 11, -(0.25 * 5 + 4.0 * 11)]  # the sink is below: sgn = -1
