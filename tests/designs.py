"""Hand-built designs for tests, in the caller format the C ABI takes.

Pure data construction: no timing arithmetic lives here.
"""
from __future__ import annotations

import numpy as np

from paper_2511_11660_amd.synth import Design

PI, CIN, COUT, PO = 0, 1, 2, 3
NX = NY = 7
SLEW_AXIS = np.array([5.0 * 60.0 ** (i / 6.0) for i in range(NX)], np.float32)
LOAD_AXIS = np.array([0.5 * 100.0 ** (j / 6.0) for j in range(NY)], np.float32)


def planar_table(a, b, c, e=0.0, xs=SLEW_AXIS, ys=LOAD_AXIS):
    """Table sampled from a + b*X + c*Y + e*X*Y on the axis grid (float32)."""
    X, Y = np.meshgrid(xs.astype(np.float64), ys.astype(np.float64), indexing="ij")
    return (a + b * X + c * Y + e * X * Y).astype(np.float32)


def make_design(pin_kind, cells, nets, n_inputs, sense, pin_cap, tables, *,
                pi_at=0.0, pi_slew=20.0, po_rat=500.0, rat_early=None, po_cap=2.0,
                dangling_policy=0, dangling_rat=None, slew_axis=None, load_axis=None):
    """cells: list of (type, [input pins], output pin).
    nets: list of dicts {driver, sinks, parent, R, C, sink_node} (RC net-local).
    tables: array [n_types, 4, NX, NY]."""
    pin_kind = np.asarray(pin_kind, np.int32)
    n_pins = len(pin_kind)
    n_pi = int((pin_kind == PI).sum())
    n_po = int((pin_kind == PO).sum())
    cell_type = np.array([c[0] for c in cells], np.int32)
    cell_in_ptr = np.zeros(len(cells) + 1, np.int32)
    for i, c in enumerate(cells):
        cell_in_ptr[i + 1] = cell_in_ptr[i] + len(c[1])
    cell_in_pin = np.array([p for c in cells for p in c[1]], np.int32)
    cell_out_pin = np.array([c[2] for c in cells], np.int32)
    net_driver = np.array([n["driver"] for n in nets], np.int32)
    net_sink_ptr = np.zeros(len(nets) + 1, np.int32)
    for i, n in enumerate(nets):
        net_sink_ptr[i + 1] = net_sink_ptr[i] + len(n["sinks"])
    net_sink_pin = np.array([s for n in nets for s in n["sinks"]], np.int32)
    net_node_ptr = np.zeros(len(nets) + 1, np.int64)
    for i, n in enumerate(nets):
        net_node_ptr[i + 1] = net_node_ptr[i] + len(n["parent"])
    parent = np.array([p for n in nets for p in n["parent"]], np.int32)
    res = np.array([r for n in nets for r in n["R"]], np.float32)
    cap = np.array([c for n in nets for c in n["C"]], np.float32)
    sink_node = np.array([k for n in nets for k in n["sink_node"]], np.int32)
    n_types = len(n_inputs)
    tables = np.asarray(tables, np.float32).reshape(n_types, 4, NX, NY)
    sa = np.tile(SLEW_AXIS if slew_axis is None else slew_axis, (n_types, 1)).astype(np.float32)
    la = np.tile(LOAD_AXIS if load_axis is None else load_axis, (n_types, 1)).astype(np.float32)
    re = po_rat if rat_early is None else rat_early
    po_rat_arr = np.tile(np.array([re, re, po_rat, po_rat], np.float32), (n_po, 1))
    dr = np.array([re, re, po_rat, po_rat], np.float32) if dangling_rat is None else \
        np.asarray(dangling_rat, np.float32)
    return Design(
        n_pins=n_pins, n_cells=len(cells), n_nets=len(nets), n_pi=n_pi, n_po=n_po,
        n_sinks=int(net_sink_ptr[-1]), n_nodes=int(net_node_ptr[-1]),
        pin_kind=pin_kind, cell_type=cell_type, cell_in_ptr=cell_in_ptr,
        cell_in_pin=cell_in_pin, cell_out_pin=cell_out_pin, net_driver=net_driver,
        net_sink_ptr=net_sink_ptr, net_sink_pin=net_sink_pin, net_node_ptr=net_node_ptr,
        parent=parent, res_kohm=res, cap_ff=cap, sink_node=sink_node,
        n_types=n_types, nx=NX, ny=NY, n_inputs=np.asarray(n_inputs, np.int32),
        sense=np.asarray(sense, np.int32), pin_cap_ff=np.asarray(pin_cap, np.float32),
        slew_axis=sa, load_axis=la, tables=tables, po_cap_ff=float(po_cap),
        pi_at=np.full((n_pi, 4), pi_at, np.float32), pi_slew=np.full((n_pi, 4), pi_slew, np.float32),
        po_rat=po_rat_arr.reshape(n_po, 4), dangling_rat=dr, dangling_policy=dangling_policy,
    )


def single_segment_net(driver, sinks, R, C):
    """Star net: each sink on its own one-segment branch from the root."""
    parent = [-1] + [0] * len(sinks)
    return {"driver": driver, "sinks": list(sinks), "parent": parent,
            "R": [0.0] + [R] * len(sinks), "C": [0.0] + [C] * len(sinks),
            "sink_node": list(range(1, len(sinks) + 1))}


def random_tree(rng, n_nodes):
    """Random rooted tree with parent[k] < k."""
    parent = [-1] + [int(rng.integers(0, k)) for k in range(1, n_nodes)]
    return parent


def tie_design():
    """Exact ties for the critical-fanin rule: a negative-unate NAND2 whose two
    inputs hang on identical branches of one net (equal arrivals and slews), a
    non-unate cell fed by a primary input whose rise and fall arrive together
    (rise and fall candidates equal), and a positive-unate AND3 whose inputs B
    and C hang on identical branches of the NAND2's output net (they tie for
    the latest arrival; input A, straight from a primary input, is earliest).

    pins: 0 PI0, 1 PI1, 2-3 NAND.A/B, 4 NAND.Y, 5 X.A, 6 X.Y, 7-9 AND.A/B/C,
    10 AND.Y, 11-12 POs."""
    kinds = [PI, PI, CIN, CIN, COUT, CIN, COUT, CIN, CIN, CIN, COUT, PO, PO]
    cells = [(0, [2, 3], 4), (1, [5], 6), (2, [7, 8, 9], 10)]
    nets = [single_segment_net(0, [2, 3], 0.02, 1.5), single_segment_net(1, [5, 7], 0.01, 0.75),
            single_segment_net(4, [8, 9], 0.03, 1.25), single_segment_net(6, [11], 0.02, 1.0),
            single_segment_net(10, [12], 0.02, 1.0)]
    tables = np.stack([
        np.stack([planar_table(9.0, 0.10, 1.3), planar_table(7.0, 0.12, 1.1),
                  planar_table(4.0, 0.05, 2.0), planar_table(3.5, 0.04, 1.9)]),
        np.stack([planar_table(6.0, 0.09, 1.0), planar_table(5.0, 0.08, 1.2),
                  planar_table(3.0, 0.04, 1.5), planar_table(2.5, 0.03, 1.6)]),
        np.stack([planar_table(11.0, 0.14, 1.4), planar_table(10.0, 0.13, 1.5),
                  planar_table(5.0, 0.06, 2.2), planar_table(4.5, 0.05, 2.1)]),
    ])
    return make_design(kinds, cells, nets, n_inputs=[2, 1, 3], sense=[1, 2, 0], pin_cap=[1.0, 1.25, 0.75],
                       tables=tables, po_rat=60.0, rat_early=5.0)
