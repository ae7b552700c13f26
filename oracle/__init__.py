"""FP64 CPU oracle (ctypes binding of ``sta_oracle.c``).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The GPU library
never loads it, and it shares no code with the GPU library.

Every function mirrors a definition of the static-timing hot path (see the
header of ``sta_oracle.c`` for the paper sections each one follows).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

_P32 = ctypes.POINTER(ctypes.c_int32)
_P64 = ctypes.POINTER(ctypes.c_int64)
_PF = ctypes.POINTER(ctypes.c_float)
_PD = ctypes.POINTER(ctypes.c_double)
_P8 = ctypes.POINTER(ctypes.c_int8)


class _ODesign(ctypes.Structure):
    _fields_ = [
        ("n_pins", ctypes.c_int32), ("n_cells", ctypes.c_int32), ("n_nets", ctypes.c_int32),
        ("n_pi", ctypes.c_int32), ("n_po", ctypes.c_int32),
        ("pin_kind", _P32),
        ("cell_type", _P32), ("cell_in_ptr", _P32), ("cell_in_pin", _P32), ("cell_out_pin", _P32),
        ("net_driver", _P32), ("net_sink_ptr", _P32), ("net_sink_pin", _P32),
        ("net_node_ptr", _P64),
        ("parent", _P32),
        ("res_kohm", _PF), ("cap_ff", _PF),
        ("sink_node", _P32),
        ("n_types", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("n_inputs", _P32), ("sense", _P32),
        ("pin_cap_ff", _PF), ("slew_axis", _PF), ("load_axis", _PF), ("tables", _PF),
        ("po_cap_ff", ctypes.c_float),
        ("pi_at", _PF), ("pi_slew", _PF), ("po_rat", _PF),
        ("dangling_rat", ctypes.c_float * 4),
        ("dangling_policy", ctypes.c_int32),
        ("res64", _PD),
        ("delay64", _PD),
        ("load64", _PD),
        ("arcd64", _PD),
    ]


class _OResult(ctypes.Structure):
    _fields_ = [
        ("level", _P32), ("level_order", _P32),
        ("L_net", _PD),
        ("d_sink", _PD), ("q_sink", _PD),
        ("at", _PD), ("slew", _PD), ("rat", _PD), ("slack", _PD),
        ("crit", _P8),
        ("ep_pin", _P32),
        ("ep_slack", _PD),
        ("ep_order", _P32),
        ("wns", ctypes.c_double * 2), ("tns", ctypes.c_double * 2),
        ("n_ep", ctypes.c_int32), ("n_levels", ctypes.c_int32),
        ("update_s", ctypes.c_double),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        lib = ctypes.CDLL(LIB_PATH)
        lib.orc_levelize.restype = ctypes.c_int
        lib.orc_levelize.argtypes = [ctypes.POINTER(_ODesign), _P32, _P32, _P32]
        lib.orc_rc.restype = None
        lib.orc_rc.argtypes = [ctypes.POINTER(_ODesign), _PD, _PD, _PD, _PD]
        lib.orc_rc_tree.restype = None
        lib.orc_rc_tree.argtypes = [ctypes.c_int64, _P32, _PD, _PD, _PD, _PD, _PD, _PD]
        lib.orc_nldm.restype = ctypes.c_double
        lib.orc_nldm.argtypes = [ctypes.c_int32, ctypes.c_int32, _PF, _PF, _PF,
                                 ctypes.c_double, ctypes.c_double]
        lib.orc_sta.restype = ctypes.c_int
        lib.orc_sta.argtypes = [ctypes.POINTER(_ODesign), _PD, ctypes.POINTER(_OResult)]
        _lib = lib
    return _lib


def _ptr(a, typ):
    return a.ctypes.data_as(typ)


class _Keep:
    """Holds the contiguous arrays a ctypes struct points into."""

    def __init__(self):
        self.arrays = []

    def __call__(self, a, dtype, typ):
        a = np.ascontiguousarray(a, dtype=dtype)
        self.arrays.append(a)
        return _ptr(a, typ)


def _odesign(d, keep: _Keep, wire_res=None, sink_delay=None, load_delta=None, arc_delta=None) -> _ODesign:
    i32 = lambda a: keep(a, np.int32, _P32)  # noqa: E731
    f32 = lambda a: keep(a, np.float32, _PF)  # noqa: E731
    od = _ODesign()
    od.n_pins, od.n_cells, od.n_nets = d.n_pins, d.n_cells, d.n_nets
    od.n_pi, od.n_po = d.n_pi, d.n_po
    od.pin_kind = i32(d.pin_kind)
    od.cell_type, od.cell_in_ptr = i32(d.cell_type), i32(d.cell_in_ptr)
    od.cell_in_pin, od.cell_out_pin = i32(d.cell_in_pin), i32(d.cell_out_pin)
    od.net_driver, od.net_sink_ptr, od.net_sink_pin = (i32(d.net_driver), i32(d.net_sink_ptr),
                                                       i32(d.net_sink_pin))
    od.net_node_ptr = keep(d.net_node_ptr, np.int64, _P64)
    od.parent = i32(d.parent)
    od.res_kohm, od.cap_ff = f32(d.res_kohm), f32(d.cap_ff)
    od.sink_node = i32(d.sink_node)
    od.n_types, od.nx, od.ny = d.n_types, d.nx, d.ny
    od.n_inputs, od.sense = i32(d.n_inputs), i32(d.sense)
    od.pin_cap_ff, od.slew_axis = f32(d.pin_cap_ff), f32(d.slew_axis)
    od.load_axis, od.tables = f32(d.load_axis), f32(d.tables)
    od.po_cap_ff = float(d.po_cap_ff)
    od.pi_at, od.pi_slew, od.po_rat = f32(d.pi_at), f32(d.pi_slew), f32(d.po_rat)
    for v in range(4):
        od.dangling_rat[v] = float(d.dangling_rat[v])
    od.dangling_policy = int(d.dangling_policy)
    od.res64 = None if wire_res is None else keep(wire_res, np.float64, _PD)
    od.delay64 = None if sink_delay is None else keep(sink_delay, np.float64, _PD)
    od.load64 = None if load_delta is None else keep(load_delta, np.float64, _PD)
    od.arcd64 = None if arc_delta is None else keep(arc_delta, np.float64, _PD)
    return od


def levelize(d):
    """Pin levels and the (level, pin id) order; raises on a cycle."""
    lib, keep = _load(), _Keep()
    od = _odesign(d, keep)
    level = np.zeros(d.n_pins, np.int32)
    order = np.zeros(d.n_pins, np.int32)
    nl = ctypes.c_int32(0)
    if lib.orc_levelize(ctypes.byref(od), _ptr(level, _P32), _ptr(order, _P32), ctypes.byref(nl)):
        raise ValueError("combinational cycle")
    return level, order, int(nl.value)


def rc(d, wire_cap=None):
    """Per net load, per sink Elmore delay d and impulse spread q (caller orders)."""
    lib, keep = _load(), _Keep()
    od = _odesign(d, keep)
    L = np.zeros(d.n_nets, np.float64)
    dd = np.zeros(d.n_sinks, np.float64)
    q = np.zeros(d.n_sinks, np.float64)
    wc = None if wire_cap is None else keep(wire_cap, np.float64, _PD)
    lib.orc_rc(ctypes.byref(od), wc, _ptr(L, _PD), _ptr(dd, _PD), _ptr(q, _PD))
    return L, dd, q


def rc_tree(parent, R, Chat):
    """Elmore recursions on one tree: (load, d, ld, m2) per node."""
    lib = _load()
    parent = np.ascontiguousarray(parent, np.int32)
    R = np.ascontiguousarray(R, np.float64)
    Chat = np.ascontiguousarray(Chat, np.float64)
    m = len(parent)
    outs = [np.zeros(m, np.float64) for _ in range(4)]
    lib.orc_rc_tree(m, _ptr(parent, _P32), _ptr(R, _PD), _ptr(Chat, _PD),
                    *[_ptr(o, _PD) for o in outs])
    return tuple(outs)


def nldm(xa, ya, table, X, Y):
    """Bilinear NLDM value with boundary-segment extrapolation."""
    lib = _load()
    xa = np.ascontiguousarray(xa, np.float32)
    ya = np.ascontiguousarray(ya, np.float32)
    table = np.ascontiguousarray(table, np.float32)
    return lib.orc_nldm(len(xa), len(ya), _ptr(xa, _PF), _ptr(ya, _PF), _ptr(table, _PF),
                        float(X), float(Y))


def sta(d, wire_cap=None, sink_delay=None):
    """Full analysis: levels, RC, AT/slew, RAT, slack, crit, endpoints, WNS/TNS.
    sink_delay (FP64, caller sink order) replaces the Elmore net delays, e.g.
    by the reduced-order delays of oracle.arnoldi.sink_delays."""
    lib, keep = _load(), _Keep()
    od = _odesign(d, keep, sink_delay=sink_delay)
    NP = d.n_pins
    r = {
        "level": np.zeros(NP, np.int32), "level_order": np.zeros(NP, np.int32),
        "L_net": np.zeros(d.n_nets, np.float64),
        "d_sink": np.zeros(max(1, d.n_sinks), np.float64),
        "q_sink": np.zeros(max(1, d.n_sinks), np.float64),
        "at": np.zeros((NP, 4), np.float64), "slew": np.zeros((NP, 4), np.float64),
        "rat": np.zeros((NP, 4), np.float64), "slack": np.zeros((NP, 4), np.float64),
        "crit": np.zeros((NP, 4), np.int8),
        "ep_pin": np.zeros(NP, np.int32),
        "ep_slack": np.zeros((NP, 2), np.float64),
        "ep_order": np.zeros(2 * NP, np.int32),
    }
    res = _OResult()
    res.level, res.level_order = _ptr(r["level"], _P32), _ptr(r["level_order"], _P32)
    res.L_net = _ptr(r["L_net"], _PD)
    res.d_sink, res.q_sink = _ptr(r["d_sink"], _PD), _ptr(r["q_sink"], _PD)
    res.at, res.slew = _ptr(r["at"], _PD), _ptr(r["slew"], _PD)
    res.rat, res.slack = _ptr(r["rat"], _PD), _ptr(r["slack"], _PD)
    res.crit = _ptr(r["crit"], _P8)
    res.ep_pin, res.ep_slack = _ptr(r["ep_pin"], _P32), _ptr(r["ep_slack"], _PD)
    res.ep_order = _ptr(r["ep_order"], _P32)
    wc = None if wire_cap is None else keep(wire_cap, np.float64, _PD)
    if lib.orc_sta(ctypes.byref(od), wc, ctypes.byref(res)):
        raise ValueError("combinational cycle")
    ne = res.n_ep
    r["n_ep"] = ne
    r["n_levels"] = res.n_levels
    r["ep_pin"] = r["ep_pin"][:ne].copy()
    r["ep_slack"] = r["ep_slack"][:ne].copy()
    r["ep_order"] = r["ep_order"][:2 * ne].reshape(2, ne).copy()
    r["d_sink"] = r["d_sink"][:d.n_sinks]
    r["q_sink"] = r["q_sink"][:d.n_sinks]
    r["wns"] = np.array([res.wns[0], res.wns[1]])
    r["tns"] = np.array([res.tns[0], res.tns[1]])
    r["update_seconds"] = res.update_s  # RC through endpoint order, without levels and pin roles
    return r


# ------------------------------------------------------------ smooth form

class _OSmooth(ctypes.Structure):
    _fields_ = [
        ("at", _PD), ("slew", _PD), ("L_net", _PD), ("d_sink", _PD), ("q_sink", _PD),
        ("ep_pin", _P32), ("ep_s", _PD),
        ("tns", ctypes.c_double), ("wns", ctypes.c_double),
        ("n_ep", ctypes.c_int32), ("sig", ctypes.c_uint64),
    ]


def _smooth_struct(d):
    NP = d.n_pins
    r = {"at": np.zeros((NP, 4)), "slew": np.zeros((NP, 4)), "L_net": np.zeros(d.n_nets),
         "d_sink": np.zeros(max(1, d.n_sinks)), "q_sink": np.zeros(max(1, d.n_sinks)),
         "ep_pin": np.zeros(NP, np.int32), "ep_s": np.zeros(NP)}
    o = _OSmooth()
    for k in ("at", "slew", "L_net", "d_sink", "q_sink", "ep_s"):
        setattr(o, k, _ptr(r[k], _PD))
    o.ep_pin = _ptr(r["ep_pin"], _P32)
    return r, o


def _smooth_finish(r, o):
    ne = o.n_ep
    r["n_ep"] = ne
    r["ep_pin"] = r["ep_pin"][:ne].copy()
    r["ep_s"] = r["ep_s"][:ne].copy()
    r["tns"], r["wns"], r["sig"] = o.tns, o.wns, o.sig
    return r


def smooth_sta(d, gamma, wire_cap=None, wire_res=None, load_delta=None, arc_delta=None):
    """Smooth forward: late AT merges by log-sum-exp (temperature gamma), smooth
    late endpoint slack, TNS_g and WNS_g.  wire_cap / wire_res (FP64, caller
    node order) override the design's node caps / segment resistances.
    load_delta [n_nets] and arc_delta [n_arcs][4] (FP64) perturb the loads the
    NLDM lookups see and the cell-arc delays, for difference checks of the
    adjoint."""
    lib, keep = _load(), _Keep()
    lib.orc_smooth_sta.restype = ctypes.c_int
    lib.orc_smooth_sta.argtypes = [ctypes.POINTER(_ODesign), _PD, ctypes.c_double, ctypes.POINTER(_OSmooth)]
    od = _odesign(d, keep, wire_res, load_delta=load_delta, arc_delta=arc_delta)
    r, o = _smooth_struct(d)
    wc = None if wire_cap is None else keep(wire_cap, np.float64, _PD)
    if lib.orc_smooth_sta(ctypes.byref(od), wc, float(gamma), ctypes.byref(o)):
        raise ValueError("combinational cycle")
    return _smooth_finish(r, o)


def smooth_adjoint(d, gamma, g_tns=1.0, g_wns=0.0, wire_cap=None, wire_res=None):
    """Gradient of g_tns*TNS_g + g_wns*WNS_g: per RC node cap and segment
    resistance (caller node order), per pin NLDM load (cell outputs), per arc
    and late view delay."""
    lib, keep = _load(), _Keep()
    lib.orc_smooth_adjoint.restype = ctypes.c_int
    lib.orc_smooth_adjoint.argtypes = [ctypes.POINTER(_ODesign), _PD, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, _PD, _PD, _PD, _PD, ctypes.POINTER(_OSmooth)]
    od = _odesign(d, keep, wire_res)
    r, o = _smooth_struct(d)
    gc = np.zeros(int(d.n_nodes))
    gr = np.zeros(int(d.n_nodes))
    gl = np.zeros(d.n_pins)
    ga = np.zeros((int(d.cell_in_ptr[-1]), 4))
    wc = None if wire_cap is None else keep(wire_cap, np.float64, _PD)
    if lib.orc_smooth_adjoint(ctypes.byref(od), wc, float(gamma), float(g_tns), float(g_wns),
                              _ptr(gc, _PD), _ptr(gr, _PD), _ptr(gl, _PD), _ptr(ga, _PD), ctypes.byref(o)):
        raise ValueError("combinational cycle")
    r = _smooth_finish(r, o)
    r["grad_wire_cap"], r["grad_wire_res"], r["grad_pin_load"], r["grad_arc_delay"] = gc, gr, gl, ga
    return r
