"""RC trees estimated from pin positions, CPU oracle.  TEST INFRASTRUCTURE ONLY
(same rule as the rest of ``oracle/``: only tests, the smoke check and the
benchmark's CPU baseline may use it).

§III "Parasitics (RC) inputs": for placement flows the timer builds each net's
RC tree itself from the pin positions and unit resistance / capacitance along
x and y (the paper runs GPU FLUTE Steiner trees for this).  FLUTE's lookup
tables are not part of the paper, so the tree here is the reading documented
with the build: a rectilinear minimum spanning tree grown by Prim's rule from
the driver, each tree edge wired as an L (along x from the parent, then along
y to the child), with the corner as an internal RC node.

Definitions (all of them are what the GPU path computes):

* pins of net n: index 0 = the driver, 1..k = the sinks in net-sink order;
* distance: |x_a - x_b| + |y_a - y_b| evaluated in FP32 (each operation
  correctly rounded), since the distances decide the tree and both sides must
  take the same decisions;
* Prim: the tree starts as {0}; every step adds the pin outside the tree with
  the smallest distance to the tree, ties to the lower pin index; its parent
  is the first tree pin (in the order pins joined) at that distance;
* the t-th pin added (t = 1..k), child c of parent p: RC node 2t-1 is the
  corner (x_c, y_p) with parent = node of p, R = r_x |x_c - x_p|,
  C = c_x |x_c - x_p|; RC node 2t is the pin, parent 2t-1, R = r_y |y_c - y_p|,
  C = c_y |y_c - y_p| (segment C lumped at the child node, the root's 0);
  node of the driver = 0, of the t-th pin = 2t;
* R and C are the FP32 roundings of the exact products of the FP32 unit
  values and FP32 lengths;
* a net of k sinks has 2k + 1 nodes; nets are laid out in net order.

Gradient to positions (``estimate_rc_backward``): with the tree held fixed, a
tree edge from parent pin p to pin c contributes R = r_x |x_c - x_p| and
C = c_x |x_c - x_p| at its corner node and the same along y at the pin node,
so dJ/dx_c gets sgn(x_c - x_p) (r_x dJ/dR + c_x dJ/dC) of the corner and
dJ/dx_p the negative, likewise along y; sgn(0) = 0 (the zero subgradient
where a segment has no length).  FP64.
"""
from __future__ import annotations

import numpy as np


def _f32(v):
    return np.float32(v)


def estimate_net(px, py, rx, ry, cx, cy):
    """One net: pins px[0], py[0] the driver, then the sinks.  Returns
    (parent [2k+1] int32 net-local, res [2k+1] float32, cap [2k+1] float32,
    node_of_pin [k+1] int32)."""
    px = np.asarray(px, np.float32)
    py = np.asarray(py, np.float32)
    k = len(px) - 1
    m = 2 * k + 1
    parent = np.full(m, -1, np.int32)
    res = np.zeros(m, np.float32)
    cap = np.zeros(m, np.float32)
    node_of = np.zeros(k + 1, np.int32)
    in_tree = np.zeros(k + 1, bool)
    in_tree[0] = True
    # float32 distances to the tree and the first tree pin that attains them
    dist = (np.abs(px - px[0]).astype(np.float32) + np.abs(py - py[0]).astype(np.float32)).astype(np.float32)
    par = np.zeros(k + 1, np.int64)
    rx64, ry64, cx64, cy64 = (float(np.float32(v)) for v in (rx, ry, cx, cy))
    for t in range(1, k + 1):
        cand = np.flatnonzero(~in_tree)
        j = int(cand[np.argmin(dist[cand])])  # argmin returns the first (lowest index) minimum
        q = int(par[j])
        lx = float(np.abs(np.float32(px[j] - px[q])))
        ly = float(np.abs(np.float32(py[j] - py[q])))
        parent[2 * t - 1] = node_of[q]
        res[2 * t - 1] = _f32(rx64 * lx)
        cap[2 * t - 1] = _f32(cx64 * lx)
        parent[2 * t] = 2 * t - 1
        res[2 * t] = _f32(ry64 * ly)
        cap[2 * t] = _f32(cy64 * ly)
        node_of[j] = 2 * t
        in_tree[j] = True
        out = np.flatnonzero(~in_tree)
        if out.size:
            dm = (np.abs((px[out] - px[j]).astype(np.float32)) + np.abs((py[out] - py[j]).astype(np.float32))).astype(
                np.float32)
            better = dm < dist[out]
            dist[out[better]] = dm[better]
            par[out[better]] = j
    return parent, res, cap, node_of


def estimate_rc(d, pin_x, pin_y, rx, ry, cx, cy):
    """RC trees of every net of design ``d`` from pin positions (caller pin
    order).  Returns a dict in the RC-CSR layout of ``sta_rc_desc``:
    net_node_ptr (int64), parent (int32, net-local, -1 at roots), res_kohm,
    cap_ff (float32) and sink_node (int32, aligned with net_sink_pin)."""
    nsp = np.asarray(d.net_sink_ptr)
    k = np.diff(nsp)
    ptr = np.zeros(d.n_nets + 1, np.int64)
    ptr[1:] = np.cumsum(2 * k + 1)
    parent = np.empty(ptr[-1], np.int32)
    res = np.empty(ptr[-1], np.float32)
    cap = np.empty(ptr[-1], np.float32)
    sink_node = np.empty(d.n_sinks, np.int32)
    pin_x = np.asarray(pin_x, np.float32)
    pin_y = np.asarray(pin_y, np.float32)
    for n in range(d.n_nets):
        pins = np.concatenate([[d.net_driver[n]], d.net_sink_pin[nsp[n]:nsp[n + 1]]])
        p, r, c, node_of = estimate_net(pin_x[pins], pin_y[pins], rx, ry, cx, cy)
        a, b = ptr[n], ptr[n + 1]
        parent[a:b], res[a:b], cap[a:b] = p, r, c
        sink_node[nsp[n]:nsp[n + 1]] = node_of[1:]
    return {"net_node_ptr": ptr, "parent": parent, "res_kohm": res, "cap_ff": cap, "sink_node": sink_node}


def estimate_rc_backward(d, pin_x, pin_y, rc, rx, ry, cx, cy, grad_res, grad_cap):
    """dJ/dx, dJ/dy per pin (FP64) from dJ/dR and dJ/dC per node of the trees
    in ``rc`` (an estimate_rc result for the same positions)."""
    x = np.asarray(pin_x, np.float64)
    y = np.asarray(pin_y, np.float64)
    gR = np.asarray(grad_res, np.float64)
    gC = np.asarray(grad_cap, np.float64)
    rx, ry, cx, cy = (float(np.float32(v)) for v in (rx, ry, cx, cy))
    gx = np.zeros(d.n_pins)
    gy = np.zeros(d.n_pins)
    nsp = np.asarray(d.net_sink_ptr)
    ptr, parent, sink_node = rc["net_node_ptr"], rc["parent"], rc["sink_node"]
    for n in range(d.n_nets):
        base = int(ptr[n])
        pin_of_node = {0: int(d.net_driver[n])}
        for s in range(nsp[n], nsp[n + 1]):
            pin_of_node[int(sink_node[s])] = int(d.net_sink_pin[s])
        for s in range(nsp[n], nsp[n + 1]):
            c = int(d.net_sink_pin[s])
            b = int(sink_node[s])
            a = b - 1
            p = pin_of_node[int(parent[base + a])]
            vx = np.sign(x[c] - x[p]) * (rx * gR[base + a] + cx * gC[base + a])
            vy = np.sign(y[c] - y[p]) * (ry * gR[base + b] + cy * gC[base + b])
            gx[c] += vx
            gx[p] -= vx
            gy[c] += vy
            gy[p] -= vy
    return gx, gy
