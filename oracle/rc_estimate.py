"""RC trees estimated from pin positions, CPU oracle.  TEST INFRASTRUCTURE ONLY
(same rule as the rest of ``oracle/``: only tests, the smoke check and the
benchmark's CPU baseline may use it).

§III "Parasitics (RC) inputs": for placement flows the timer builds each net's
RC tree itself from the pin positions and unit resistance / capacitance along
x and y, as rectilinear Steiner trees (the paper runs GPU FLUTE for this).
FLUTE's lookup tables are not part of the paper, so the Steiner tree here is
the reading documented with the build: the shortest-path heuristic of
Takahashi and Matsuyama (1980) taken to the rectilinear plane.  The tree
starts as the driver alone; every step joins the pin outside the tree that is
nearest to the tree's WIRES (not only to its pins), along an L from the
nearest point of the nearest wire.  Where that point lies inside a wire, the
wire is split there and the new branch leaves from a Steiner point.

Definitions (all of them are what the GPU path computes):

* pins of net n: index 0 = the driver, 1..k = the sinks in net-sink order;
* wires ("segments"): segment 0 is the driver's point; step t (t = 1..k)
  adds segment 2t-1, along x from the attach point q_t to the corner
  K_t = (x_j, q_t.y), and segment 2t, along y from K_t to the pin j;
* distance of pin u to a segment: |x_u - c_x| + |y_u - c_y| in FP32, with c
  the segment's point nearest to u: the segment's fixed coordinate and u's
  other coordinate clamped to the segment's range (clamp(v, lo, hi) = lo if
  v < lo, hi if v > hi, else v; lo / hi the smaller / larger end);
* every pin outside the tree keeps its smallest distance and the segment and
  point that give it; a new segment replaces them only if strictly nearer
  (2t-1 is tried before 2t), so ties stay with the older segment;
* step t joins the pin with the smallest distance, ties to the lower pin
  index; its recorded point is q_t and its segment sigma_t;
* RC nodes: the driver D, and per step t the Steiner point S_t (at q_t on
  sigma_t), the corner K_t and the pin J_t.  Along each segment the points
  on it (its start, the S of every step attached to it, its end) form a
  chain ordered by distance from the start (ties by step); each point's
  parent is the previous one.  The start of 2t-1 is S_t, of 2t is K_t; the
  end of 2t-1 is K_t, of 2t is J_t; segment 0 is D followed by its S points;
* node numbering: segments in order 0, 1, ..., 2k, each contributing its
  chain without the start (segment 0: D first); within a segment, its S
  points in chain order, then its end.  A start always lies on an earlier
  segment, so every parent precedes its child; the net has 3k + 1 nodes;
* a node's R and C are the unit values of its segment's axis times its
  distance to its parent (|difference of the coordinate along the axis|,
  FP32), C lumped at the node; the driver's are 0.

Gradient to positions (``estimate_rc_backward``): with the tree held fixed,
every node coordinate is a copy of some pin's coordinate (a clamp picks one
of its three candidates), so a piece of length |c_u - c_w| along x adds
sgn(c_u - c_w) (r_x dJ/dR + c_x dJ/dC) of node u to dJ/dx of the pin that
c_u copies and the negative to the pin c_w copies; likewise along y;
sgn(0) = 0.  FP64.
"""
from __future__ import annotations

import numpy as np

_F = np.float32


def sph_net(px, py):
    """The join sequence of one net.  Returns a list of steps (t = 1..k), each
    a dict: j (pin), sigma (segment attached to), q = (qx, qy), and the
    source pins of qx and qy.  The per-pin relaxation runs over numpy FP32
    arrays (elementwise, the same operations as the scalar definition)."""
    px = np.asarray(px, _F)
    py = np.asarray(py, _F)
    k = len(px) - 1
    u = np.arange(k + 1)
    dist = (np.abs(px - px[0]) + np.abs(py - py[0])).astype(_F)
    seg = np.zeros(k + 1, np.int64)
    ncx = np.full(k + 1, px[0], _F)
    ncy = np.full(k + 1, py[0], _F)
    scx = np.zeros(k + 1, np.int64)
    scy = np.zeros(k + 1, np.int64)
    live = np.ones(k + 1, bool)
    live[0] = False
    steps = []
    for t in range(1, k + 1):
        cand = np.flatnonzero(live)
        j = int(cand[np.argmin(dist[cand])])  # the first (lowest index) minimum
        qx, qy, sqx, sqy = ncx[j], ncy[j], int(scx[j]), int(scy[j])
        steps.append({"j": j, "sigma": int(seg[j]), "q": (qx, qy), "src": (sqx, sqy)})
        live[j] = False
        # segment 2t-1: y = qy, x from qx to x_j; segment 2t: x = x_j, y from qy to y_j
        for s, along_x, f, sf, a, sa, b, sb in ((2 * t - 1, True, qy, sqy, qx, sqx, px[j], j),
                                                (2 * t, False, px[j], j, qy, sqy, py[j], j)):
            lo, slo, hi, shi = (a, sa, b, sb) if not (b < a) else (b, sb, a, sa)
            v = px if along_x else py
            c = np.where(v < lo, lo, np.where(v > hi, hi, v)).astype(_F)
            sc = np.where(v < lo, slo, np.where(v > hi, shi, u))
            cx, cy = (c, np.full(k + 1, f, _F)) if along_x else (np.full(k + 1, f, _F), c)
            d = (np.abs(px - cx) + np.abs(py - cy)).astype(_F)
            up = live & (d < dist)
            dist[up] = d[up]
            seg[up] = s
            ncx[up] = cx[up]
            ncy[up] = cy[up]
            if along_x:
                scx[up] = sc[up]
                scy[up] = sf
            else:
                scx[up] = sf
                scy[up] = sc[up]
    return steps


def build_net(px, py, rx, ry, cx, cy, steps=None):
    """RC tree of one net.  Returns (parent [3k+1] int32 net-local, res, cap
    [3k+1] float32, node_of_pin [k+1] int32, src [3k+1, 2] int32: the pins
    whose x and y each node copies, axis [3k+1] int8: 0 where a node's piece
    runs along x, 1 along y, -1 at the root)."""
    px = np.asarray(px, _F)
    py = np.asarray(py, _F)
    k = len(px) - 1
    if steps is None:
        steps = sph_net(px, py)
    m = 3 * k + 1
    # node positions and coordinate sources, by role: D, and S_t, K_t, J_t
    pos = {("D", 0): (px[0], py[0], 0, 0)}
    for t, st in enumerate(steps, 1):
        j = st["j"]
        qx, qy = st["q"]
        sqx, sqy = st["src"]
        pos[("S", t)] = (qx, qy, sqx, sqy)
        pos[("K", t)] = (px[j], qy, j, sqy)
        pos[("J", t)] = (px[j], py[j], j, j)
    # each segment: axis, start node, end node
    seg = {0: ("x", ("D", 0), None)}
    for t in range(1, k + 1):
        seg[2 * t - 1] = ("x", ("S", t), ("K", t))
        seg[2 * t] = ("y", ("K", t), ("J", t))

    def coord(node, axis):
        p = pos[node]
        return p[0] if axis == "x" else p[1]

    # chain of each segment: its S points ordered by distance from the start
    # (the coordinate times the segment's direction), ties by step
    chains = {s: [] for s in seg}
    for t, st in enumerate(steps, 1):
        chains[st["sigma"]].append(t)
    order = []  # node numbering
    parent_of = {}
    axis_of = {}
    for s in range(2 * k + 1):
        axis, start, end = seg[s]
        c0 = coord(start, axis)
        dirn = _F(-1.0) if (end is not None and coord(end, axis) < c0) else _F(1.0)
        ch = sorted(chains[s], key=lambda t: (_F(dirn * coord(("S", t), axis)), t))
        if s == 0:
            order.append(start)
        prev = start
        for t in ch:
            parent_of[("S", t)] = prev
            axis_of[("S", t)] = axis
            order.append(("S", t))
            prev = ("S", t)
        if end is not None:
            parent_of[end] = prev
            axis_of[end] = axis
            order.append(end)
    assert len(order) == m
    index = {node: i for i, node in enumerate(order)}
    parent = np.full(m, -1, np.int32)
    res = np.zeros(m, _F)
    cap = np.zeros(m, _F)
    src = np.zeros((m, 2), np.int32)
    ax = np.full(m, -1, np.int8)
    r = {"x": float(_F(rx)), "y": float(_F(ry))}
    c = {"x": float(_F(cx)), "y": float(_F(cy))}
    for node, i in index.items():
        p = pos[node]
        src[i] = (p[2], p[3])
        if node == ("D", 0):
            continue
        w = parent_of[node]
        a = axis_of[node]
        L = float(abs(_F(coord(node, a) - coord(w, a))))
        parent[i] = index[w]
        ax[i] = 0 if a == "x" else 1
        res[i] = _F(r[a] * L)  # the FP32 rounding of the exact product
        cap[i] = _F(c[a] * L)
    node_of = np.zeros(k + 1, np.int32)
    for t, st in enumerate(steps, 1):
        node_of[st["j"]] = index[("J", t)]
    return parent, res, cap, node_of, src, ax


def estimate_net(px, py, rx, ry, cx, cy):
    """One net: pins px[0], py[0] the driver, then the sinks.  Returns
    (parent [3k+1] int32 net-local, res [3k+1] float32, cap [3k+1] float32,
    node_of_pin [k+1] int32)."""
    parent, res, cap, node_of, _, _ = build_net(px, py, rx, ry, cx, cy)
    return parent, res, cap, node_of


def _net_pins(d, n):
    nsp = np.asarray(d.net_sink_ptr)
    return np.concatenate([[d.net_driver[n]], d.net_sink_pin[nsp[n]:nsp[n + 1]]]).astype(np.int64)


def estimate_rc(d, pin_x, pin_y, rx, ry, cx, cy):
    """RC trees of every net of design ``d`` from pin positions (caller pin
    order).  Returns a dict in the RC-CSR layout of ``sta_rc_desc``:
    net_node_ptr (int64), parent (int32, net-local, -1 at roots), res_kohm,
    cap_ff (float32) and sink_node (int32, aligned with net_sink_pin)."""
    nsp = np.asarray(d.net_sink_ptr)
    k = np.diff(nsp)
    ptr = np.zeros(d.n_nets + 1, np.int64)
    ptr[1:] = np.cumsum(3 * k + 1)
    parent = np.empty(ptr[-1], np.int32)
    res = np.empty(ptr[-1], np.float32)
    cap = np.empty(ptr[-1], np.float32)
    sink_node = np.empty(d.n_sinks, np.int32)
    pin_x = np.asarray(pin_x, np.float32)
    pin_y = np.asarray(pin_y, np.float32)
    for n in range(d.n_nets):
        pins = _net_pins(d, n)
        p, r, c, node_of = estimate_net(pin_x[pins], pin_y[pins], rx, ry, cx, cy)
        a, b = ptr[n], ptr[n + 1]
        parent[a:b], res[a:b], cap[a:b] = p, r, c
        sink_node[nsp[n]:nsp[n + 1]] = node_of[1:]
    return {"net_node_ptr": ptr, "parent": parent, "res_kohm": res, "cap_ff": cap, "sink_node": sink_node}


def estimate_rc_backward(d, pin_x, pin_y, rc, rx, ry, cx, cy, grad_res, grad_cap):
    """dJ/dx, dJ/dy per pin (FP64) from dJ/dR and dJ/dC per node of the trees
    in ``rc`` (an estimate_rc result for the same positions: the trees are
    rebuilt from the positions and must match it)."""
    x = np.asarray(pin_x, np.float32)
    y = np.asarray(pin_y, np.float32)
    gR = np.asarray(grad_res, np.float64)
    gC = np.asarray(grad_cap, np.float64)
    r = {0: float(np.float32(rx)), 1: float(np.float32(ry))}
    c = {0: float(np.float32(cx)), 1: float(np.float32(cy))}
    gx = np.zeros(d.n_pins)
    gy = np.zeros(d.n_pins)
    nsp = np.asarray(d.net_sink_ptr)
    ptr = rc["net_node_ptr"]
    for n in range(d.n_nets):
        pins = _net_pins(d, n)
        px, py = x[pins], y[pins]
        parent, res, cap, node_of, src, ax = build_net(px, py, rx, ry, cx, cy)
        base = int(ptr[n])
        assert np.array_equal(parent, rc["parent"][base:base + parent.size])
        assert np.array_equal(node_of[1:], rc["sink_node"][nsp[n]:nsp[n + 1]])
        for i in range(1, parent.size):
            a = int(ax[i])
            coords, g = ((px, gx), (py, gy))[a]
            su, sw = int(src[i, a]), int(src[parent[i], a])
            v = np.sign(float(coords[su]) - float(coords[sw])) * (r[a] * gR[base + i] + c[a] * gC[base + i])
            g[pins[su]] += v
            g[pins[sw]] -= v
    return gx, gy
