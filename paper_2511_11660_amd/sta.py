"""ctypes binding of ``libsta.so`` (declared in ``include/sta.h``).

The module-level functions carry the C names and only marshal arguments:
every step of the timing path runs in the library's HIP kernels.  Host
arrays are numpy; device arrays are anything exposing ``data_ptr()`` (torch
tensors on ``cuda``), and streams are raw HIP stream handles (an int) or a
torch stream.  ``STA`` is a small owner of one context built from a
``synth.Design``-shaped object.

There is no CPU fallback: if ``libsta.so`` is missing or fails to load, every
entry point raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsta.so")

STA_OK, STA_E_ARG, STA_E_CYCLE, STA_E_OOM, STA_E_DEVICE, STA_E_STATE, STA_E_UNSUPPORTED = range(7)
STA_HOST, STA_DEVICE = 0, 1
STA_SCHED_PERSISTENT, STA_SCHED_PER_LEVEL, STA_SCHED_GRAPH, STA_SCHED_FLOW = 0, 1, 2, 3

_P32 = ctypes.POINTER(ctypes.c_int32)
_P64 = ctypes.POINTER(ctypes.c_int64)
_PF = ctypes.POINTER(ctypes.c_float)
_PD = ctypes.POINTER(ctypes.c_double)
_VP = ctypes.c_void_p


class sta_graph_desc(ctypes.Structure):
    _fields_ = [("n_pins", ctypes.c_int32), ("n_cells", ctypes.c_int32), ("n_nets", ctypes.c_int32),
                ("n_pi", ctypes.c_int32), ("n_po", ctypes.c_int32),
                ("pin_kind", _VP), ("cell_type", _VP), ("cell_in_ptr", _VP), ("cell_in_pin", _VP),
                ("cell_out_pin", _VP), ("net_driver", _VP), ("net_sink_ptr", _VP),
                ("net_sink_pin", _VP), ("mem", ctypes.c_int)]


class sta_rc_desc(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int64), ("net_node_ptr", _VP), ("parent", _VP),
                ("res_kohm", _VP), ("cap_ff", _VP), ("sink_node", _VP), ("mem", ctypes.c_int)]


class sta_lib_desc(ctypes.Structure):
    _fields_ = [("n_types", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("n_inputs", _VP), ("sense", _VP), ("pin_cap_ff", _VP), ("slew_axis", _VP),
                ("load_axis", _VP), ("tables", _VP), ("po_cap_ff", ctypes.c_float)]


class sta_constraints(ctypes.Structure):
    _fields_ = [("pi_at", _VP), ("pi_slew", _VP), ("po_rat", _VP),
                ("dangling_rat", ctypes.c_float * 4)]


class sta_options(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("gamma_ps", ctypes.c_float),
                ("dangling_policy", ctypes.c_int32), ("sched", ctypes.c_int32),
                ("big_net_nodes", ctypes.c_int32), ("sort_endpoints", ctypes.c_int32),
                ("profile", ctypes.c_int32), ("device", ctypes.c_int32), ("sweep_blocks", ctypes.c_int32),
                ("delay_model", ctypes.c_int32), ("overlap", ctypes.c_int32)]


class sta_info(ctypes.Structure):
    _fields_ = [("n_pins", ctypes.c_int32), ("n_cells", ctypes.c_int32), ("n_nets", ctypes.c_int32),
                ("n_pi", ctypes.c_int32), ("n_po", ctypes.c_int32), ("n_sinks", ctypes.c_int32),
                ("n_nodes", ctypes.c_int64), ("n_levels", ctypes.c_int32),
                ("n_cell_levels", ctypes.c_int32), ("n_endpoints", ctypes.c_int32),
                ("n_big_nets", ctypes.c_int32), ("n_chunks", ctypes.c_int32),
                ("device", ctypes.c_int32)]


class sta_tune_result(ctypes.Structure):
    _fields_ = [("sched", ctypes.c_int32), ("sweep_blocks", ctypes.c_int32), ("ms", ctypes.c_float),
                ("n_tried", ctypes.c_int32), ("overlap", ctypes.c_int32)]


class sta_path_query(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("per_endpoint", ctypes.c_int32), ("slack_below", ctypes.c_float),
                ("el", ctypes.c_int32)]


class sta_wire_params(ctypes.Structure):
    _fields_ = [("r_x", ctypes.c_float), ("r_y", ctypes.c_float), ("c_x", ctypes.c_float),
                ("c_y", ctypes.c_float)]


# (name, restype, argtypes) of every exported function
_SIGS = [
    ("sta_options_default", None, [ctypes.POINTER(sta_options)]),
    ("sta_create", ctypes.c_int, [ctypes.POINTER(sta_graph_desc), ctypes.POINTER(sta_rc_desc),
                                  ctypes.POINTER(sta_lib_desc), ctypes.POINTER(sta_constraints),
                                  ctypes.POINTER(sta_options), ctypes.POINTER(_VP)]),
    ("sta_destroy", None, [_VP]),
    ("sta_set_wire_caps", ctypes.c_int, [_VP, _VP, ctypes.c_int, _VP]),
    ("sta_update_timing", ctypes.c_int, [_VP, _VP]),
    ("sta_update_timing_incremental", ctypes.c_int, [_VP, _VP, ctypes.c_int32, ctypes.c_int, _VP]),
    ("sta_report_slack", ctypes.c_int, [_VP, _VP, _VP, _VP, _PD, _PD, ctypes.c_int, _VP]),
    ("sta_report_timing", ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, ctypes.c_int, _VP]),
    ("sta_report_levels", ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int, _VP]),
    ("sta_report_rc", ctypes.c_int, [_VP, _VP, _VP, _VP, ctypes.c_int, _VP]),
    ("sta_report_endpoints", ctypes.c_int, [_VP, _VP, ctypes.c_int, _VP]),
    ("sta_get_info", ctypes.c_int, [_VP, ctypes.POINTER(sta_info)]),
    ("sta_get_phase_times", ctypes.c_int, [_VP, _PF, _P32]),
    ("sta_backward", ctypes.c_int, [_VP, ctypes.c_float, ctypes.c_float, _VP, _VP, _VP, _VP, ctypes.c_int, _VP]),
    ("sta_batch_create", ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(sta_graph_desc),
                                        ctypes.POINTER(sta_rc_desc), ctypes.POINTER(sta_lib_desc),
                                        ctypes.POINTER(sta_constraints), ctypes.POINTER(sta_options),
                                        ctypes.POINTER(_VP)]),
    ("sta_batch_create_libs", ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(sta_graph_desc),
                                             ctypes.POINTER(sta_rc_desc), ctypes.POINTER(ctypes.POINTER(sta_lib_desc)),
                                             ctypes.POINTER(sta_constraints), ctypes.POINTER(sta_options),
                                             ctypes.POINTER(_VP)]),
    ("sta_batch_offsets", ctypes.c_int, [_VP, _P32, _P32, _P32, _P64]),
    ("sta_batch_report", ctypes.c_int, [_VP, _PD, _PD, _VP]),
    ("sta_autotune", ctypes.c_int, [_VP, ctypes.c_int32, ctypes.POINTER(sta_tune_result), _VP]),
    ("sta_report_paths", ctypes.c_int, [_VP, ctypes.POINTER(sta_path_query), _P32, _VP, _VP, _VP, _VP, _VP,
                                        ctypes.c_int, _VP]),
    ("sta_estimate_rc", ctypes.c_int, [ctypes.POINTER(sta_graph_desc), _VP, _VP, ctypes.POINTER(sta_wire_params),
                                       _VP, _VP, _VP, _VP, _VP, ctypes.c_int, _VP]),
    ("sta_measure_copy", ctypes.c_int, [_VP, _VP, ctypes.c_int64, ctypes.c_int32, _VP, _PF]),
    ("sta_measure_level_floor", ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32,
                                               _VP, _PF]),
    ("sta_estimate_rc_noalloc", ctypes.c_int, [ctypes.POINTER(sta_graph_desc), _VP, _VP,
                                               ctypes.POINTER(sta_wire_params), _VP, _VP, _VP, _VP, _VP, _VP]),
    ("sta_estimate_rc_backward", ctypes.c_int, [ctypes.POINTER(sta_graph_desc), _VP, _VP,
                                                ctypes.POINTER(sta_wire_params), _VP, _VP, _VP, _VP, _VP, _VP,
                                                ctypes.c_int, _VP]),
    ("sta_status_string", ctypes.c_char_p, [ctypes.c_int]),
    ("sta_last_error", ctypes.c_char_p, []),
]

_lib = None
_hip = None


def hip_runtime_path() -> str:
    """The HIP runtime this process uses: torch's bundled copy when torch is
    importable (so device pointers, streams and the device state are shared
    with torch), else the system ROCm runtime."""
    try:
        import torch
        p = os.path.join(os.path.dirname(torch.__file__), "lib", "libamdhip64.so")
        if os.path.exists(p):
            return p
    except ImportError:
        pass
    for p in ("/opt/rocm/lib/libamdhip64.so.7", "/opt/rocm/lib/libamdhip64.so"):
        if os.path.exists(p):
            return p
    raise RuntimeError("no HIP runtime found")


def load() -> ctypes.CDLL:
    """Loads libsta.so (raises if it is not built).  The HIP runtime is loaded
    first into the global symbol scope; libsta.so binds to it."""
    global _lib, _hip
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        _hip = ctypes.CDLL(hip_runtime_path(), mode=ctypes.RTLD_GLOBAL)
        lib = ctypes.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


class StaError(RuntimeError):
    def __init__(self, status: int, msg: str):
        self.status = status
        super().__init__(f"{sta_status_string(status)}: {msg}")


def sta_status_string(s: int) -> str:
    return load().sta_status_string(s).decode()


def sta_last_error() -> str:
    return load().sta_last_error().decode()


def _check(status: int) -> None:
    if status != STA_OK:
        raise StaError(status, sta_last_error())


def _addr(a) -> int | None:
    """Address of a numpy array / torch tensor / int, or None."""
    if a is None:
        return None
    if isinstance(a, int):
        return a
    if hasattr(a, "data_ptr"):
        return a.data_ptr()
    if isinstance(a, np.ndarray):
        if not a.flags["C_CONTIGUOUS"]:
            raise ValueError("array must be C-contiguous")
        return a.ctypes.data
    raise TypeError(f"cannot take the address of {type(a)}")


def _stream(s) -> int | None:
    if s is None:
        return None
    if isinstance(s, int):
        return s
    return s.cuda_stream  # torch.cuda.Stream


def sta_options_default() -> sta_options:
    o = sta_options()
    load().sta_options_default(ctypes.byref(o))
    return o


def sta_create(graph: sta_graph_desc, rc: sta_rc_desc, lib: sta_lib_desc, cons: sta_constraints,
               opts: sta_options | None = None) -> int:
    ctx = _VP()
    _check(load().sta_create(ctypes.byref(graph), ctypes.byref(rc), ctypes.byref(lib),
                             ctypes.byref(cons), ctypes.byref(opts) if opts is not None else None,
                             ctypes.byref(ctx)))
    return ctx.value


def sta_destroy(ctx: int) -> None:
    load().sta_destroy(ctx)


def sta_set_wire_caps(ctx: int, cap_ff, mem: int, stream=None) -> None:
    _check(load().sta_set_wire_caps(ctx, _addr(cap_ff), mem, _stream(stream)))


def sta_update_timing(ctx: int, stream=None) -> None:
    _check(load().sta_update_timing(ctx, _stream(stream)))


def sta_update_timing_incremental(ctx: int, nets, mem: int = STA_HOST, stream=None) -> None:
    if nets is None:
        _check(load().sta_update_timing_incremental(ctx, None, 0, mem, _stream(stream)))
        return
    if mem == STA_HOST:
        nets = np.ascontiguousarray(nets, np.int32)
    n = int(nets.shape[0]) if hasattr(nets, "shape") else len(nets)
    _check(load().sta_update_timing_incremental(ctx, _addr(nets) if n else None, n, mem, _stream(stream)))


def sta_report_slack(ctx: int, pin_slack=None, ep_slack=None, ep_order=None, dst: int = STA_HOST,
                     stream=None):
    wns = (ctypes.c_double * 2)()
    tns = (ctypes.c_double * 2)()
    _check(load().sta_report_slack(ctx, _addr(pin_slack), _addr(ep_slack), _addr(ep_order),
                                   ctypes.cast(wns, _PD), ctypes.cast(tns, _PD), dst, _stream(stream)))
    return np.array(list(wns)), np.array(list(tns))


def sta_report_timing(ctx: int, at=None, slew=None, rat=None, crit=None, dst: int = STA_HOST,
                      stream=None) -> None:
    _check(load().sta_report_timing(ctx, _addr(at), _addr(slew), _addr(rat), _addr(crit), dst,
                                    _stream(stream)))


def sta_report_levels(ctx: int, pin_level=None, level_order=None, dst: int = STA_HOST,
                      stream=None) -> None:
    _check(load().sta_report_levels(ctx, _addr(pin_level), _addr(level_order), dst, _stream(stream)))


def sta_report_rc(ctx: int, net_load=None, sink_delay=None, sink_spread=None, dst: int = STA_HOST,
                  stream=None) -> None:
    _check(load().sta_report_rc(ctx, _addr(net_load), _addr(sink_delay), _addr(sink_spread), dst,
                                _stream(stream)))


def sta_report_endpoints(ctx: int, ep_pin=None, dst: int = STA_HOST, stream=None) -> None:
    _check(load().sta_report_endpoints(ctx, _addr(ep_pin), dst, _stream(stream)))


def sta_get_info(ctx: int) -> sta_info:
    info = sta_info()
    _check(load().sta_get_info(ctx, ctypes.byref(info)))
    return info


def sta_get_phase_times(ctx: int) -> np.ndarray:
    ms = (ctypes.c_float * 8)()
    n = ctypes.c_int32(0)
    _check(load().sta_get_phase_times(ctx, ctypes.cast(ms, _PF), ctypes.byref(n)))
    return np.array(list(ms)[: n.value], dtype=np.float64)


def sta_backward(ctx: int, g_tns: float, g_wns: float, grad_wire_cap=None, grad_wire_res=None, grad_pin_load=None,
                 grad_arc_delay=None, dst: int = STA_HOST, stream=None) -> None:
    _check(load().sta_backward(ctx, float(g_tns), float(g_wns), _addr(grad_wire_cap), _addr(grad_wire_res),
                               _addr(grad_pin_load), _addr(grad_arc_delay), dst, _stream(stream)))


def sta_batch_create(graphs, rcs, lib: sta_lib_desc, cons, opts: sta_options | None = None) -> int:
    n = len(graphs)
    if not (len(rcs) == len(cons) == n):
        raise ValueError("graphs, rcs and cons must have one entry per design")
    ga = (sta_graph_desc * n)(*graphs)
    ra = (sta_rc_desc * n)(*rcs)
    ca = (sta_constraints * n)(*cons)
    ctx = _VP()
    _check(load().sta_batch_create(n, ga, ra, ctypes.byref(lib), ca,
                                   ctypes.byref(opts) if opts is not None else None, ctypes.byref(ctx)))
    return ctx.value


def sta_batch_create_libs(graphs, rcs, libs, cons, opts: sta_options | None = None) -> int:
    """Batch with one library per design; equal entries of libs (the same
    sta_lib_desc object) share one library."""
    n = len(graphs)
    if not (len(rcs) == len(cons) == len(libs) == n):
        raise ValueError("graphs, rcs, libs and cons must have one entry per design")
    ga = (sta_graph_desc * n)(*graphs)
    ra = (sta_rc_desc * n)(*rcs)
    ca = (sta_constraints * n)(*cons)
    la = (ctypes.POINTER(sta_lib_desc) * n)(*[ctypes.pointer(l) for l in libs])
    ctx = _VP()
    _check(load().sta_batch_create_libs(n, ga, ra, la, ca, ctypes.byref(opts) if opts is not None else None,
                                        ctypes.byref(ctx)))
    return ctx.value


def sta_batch_offsets(ctx: int):
    """(pin_off, ep_off, node_off) numpy arrays of n_designs + 1 entries."""
    n = ctypes.c_int32(0)
    _check(load().sta_batch_offsets(ctx, ctypes.byref(n), None, None, None))
    pin = np.zeros(n.value + 1, np.int32)
    ep = np.zeros(n.value + 1, np.int32)
    node = np.zeros(n.value + 1, np.int64)
    _check(load().sta_batch_offsets(ctx, ctypes.byref(n), pin.ctypes.data_as(_P32), ep.ctypes.data_as(_P32),
                                    node.ctypes.data_as(_P64)))
    return pin, ep, node


def sta_batch_report(ctx: int, n_designs: int, stream=None):
    """Per-design (wns, tns), each [n_designs][2] (early, late)."""
    wns = np.zeros((n_designs, 2), np.float64)
    tns = np.zeros((n_designs, 2), np.float64)
    _check(load().sta_batch_report(ctx, wns.ctypes.data_as(_PD), tns.ctypes.data_as(_PD), _stream(stream)))
    return wns, tns


def sta_autotune(ctx: int, reps: int = 5, stream=None) -> sta_tune_result:
    r = sta_tune_result()
    _check(load().sta_autotune(ctx, int(reps), ctypes.byref(r), _stream(stream)))
    return r


def sta_report_paths(ctx: int, k: int, per_endpoint: int = 1, slack_below: float = float("inf"), el: int = 1,
                     max_len: int = 0, stream=None):
    """Top-k path report into host arrays; returns a list of dicts (slack,
    endpoint index, pins and transitions from startpoint to endpoint)."""
    q = sta_path_query(int(k), int(per_endpoint), float(slack_below), int(el))
    if max_len <= 0:
        max_len = sta_get_info(ctx).n_levels
    n = ctypes.c_int32(0)
    ptr = np.zeros(k + 1, np.int32)
    pins = np.zeros(k * max_len, np.int32)
    rf = np.zeros(k * max_len, np.int8)
    slack = np.zeros(k, np.float32)
    ep = np.zeros(k, np.int32)
    _check(load().sta_report_paths(ctx, ctypes.byref(q), ctypes.byref(n), _addr(ptr), _addr(pins), _addr(rf),
                                   _addr(slack), _addr(ep), STA_HOST, _stream(stream)))
    out = []
    for i in range(n.value):
        a, b = ptr[i], ptr[i + 1]
        out.append({"slack": float(slack[i]), "endpoint": int(ep[i]), "pins": pins[a:b].tolist(),
                    "rf": rf[a:b].tolist()})
    return out


def sta_estimate_rc(graph: sta_graph_desc, pin_x, pin_y, wire: sta_wire_params, net_node_ptr, parent, res_kohm,
                    cap_ff, sink_node, mem: int = STA_HOST, stream=None) -> None:
    _check(load().sta_estimate_rc(ctypes.byref(graph), _addr(pin_x), _addr(pin_y), ctypes.byref(wire),
                                  _addr(net_node_ptr), _addr(parent), _addr(res_kohm), _addr(cap_ff),
                                  _addr(sink_node), mem, _stream(stream)))


def sta_measure_copy(src, dst, nbytes: int, reps: int = 10, stream=None) -> float:
    """Mean ms of one plain device copy of nbytes from src to dst."""
    ms = ctypes.c_float(0.0)
    _check(load().sta_measure_copy(_addr(src), _addr(dst), int(nbytes), int(reps), _stream(stream), ctypes.byref(ms)))
    return ms.value


def sta_measure_level_floor(levels: int, items: int, records: int, reps: int = 5, stream=None) -> float:
    """Mean ms of `levels` dependent level-shaped launches (see sta.h)."""
    ms = ctypes.c_float(0.0)
    _check(load().sta_measure_level_floor(int(levels), int(items), int(records), int(reps), _stream(stream),
                                          ctypes.byref(ms)))
    return ms.value


def sta_estimate_rc_noalloc(graph: sta_graph_desc, pin_x, pin_y, wire: sta_wire_params, net_node_ptr, parent,
                            res_kohm, cap_ff, sink_node, stream=None) -> None:
    _check(load().sta_estimate_rc_noalloc(ctypes.byref(graph), _addr(pin_x), _addr(pin_y), ctypes.byref(wire),
                                          _addr(net_node_ptr), _addr(parent), _addr(res_kohm), _addr(cap_ff),
                                          _addr(sink_node), _stream(stream)))


def estimate_rc(d, pin_x, pin_y, r_x, r_y, c_x, c_y, stream=None) -> dict:
    """RC trees of every net of a synth.Design-shaped object from pin
    positions, as host arrays in the RC-CSR layout (keys as in synth.Design:
    net_node_ptr, parent, res_kohm, cap_ff, sink_node).  Positions may be
    numpy arrays (host) or cuda tensors (device; outputs are then cuda tensors
    too)."""
    keep: list = []

    def a(x, dt):
        x = np.ascontiguousarray(x, dtype=dt)
        keep.append(x)
        return x.ctypes.data

    g = sta_graph_desc(d.n_pins, d.n_cells, d.n_nets, d.n_pi, d.n_po, None, None, None, None, None,
                       a(d.net_driver, np.int32), a(d.net_sink_ptr, np.int32),
                       a(d.net_sink_pin, np.int32), STA_HOST)
    n_sinks = int(np.asarray(d.net_sink_ptr)[-1])
    n_nodes = d.n_nets + 3 * n_sinks
    w = sta_wire_params(r_x, r_y, c_x, c_y)
    if hasattr(pin_x, "data_ptr"):
        import torch
        dev = pin_x.device
        pin_x = pin_x.contiguous().float()
        pin_y = pin_y.contiguous().float()
        out = {"net_node_ptr": torch.empty(d.n_nets + 1, dtype=torch.int64, device=dev),
               "parent": torch.empty(max(n_nodes, 1), dtype=torch.int32, device=dev),
               "res_kohm": torch.empty(max(n_nodes, 1), dtype=torch.float32, device=dev),
               "cap_ff": torch.empty(max(n_nodes, 1), dtype=torch.float32, device=dev),
               "sink_node": torch.empty(max(n_sinks, 1), dtype=torch.int32, device=dev)}
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        mem = STA_DEVICE
    else:
        pin_x = np.ascontiguousarray(pin_x, np.float32)
        pin_y = np.ascontiguousarray(pin_y, np.float32)
        out = {"net_node_ptr": np.zeros(d.n_nets + 1, np.int64), "parent": np.zeros(n_nodes, np.int32),
               "res_kohm": np.zeros(n_nodes, np.float32), "cap_ff": np.zeros(n_nodes, np.float32),
               "sink_node": np.zeros(n_sinks, np.int32)}
        mem = STA_HOST
    sta_estimate_rc(g, pin_x, pin_y, w, out["net_node_ptr"], out["parent"], out["res_kohm"], out["cap_ff"],
                    out["sink_node"], mem, stream)
    if mem == STA_DEVICE:
        out = {k: (v[:n_nodes] if k in ("parent", "res_kohm", "cap_ff") else v) for k, v in out.items()}
        out["sink_node"] = out["sink_node"][:n_sinks]
    return out


def sta_estimate_rc_backward(graph: sta_graph_desc, pin_x, pin_y, wire: sta_wire_params, parent, sink_node,
                             grad_res, grad_cap, grad_x, grad_y, mem: int = STA_HOST, stream=None) -> None:
    _check(load().sta_estimate_rc_backward(ctypes.byref(graph), _addr(pin_x), _addr(pin_y), ctypes.byref(wire),
                                           _addr(parent), _addr(sink_node), _addr(grad_res), _addr(grad_cap),
                                           _addr(grad_x), _addr(grad_y), mem, _stream(stream)))


def _net_graph(d, keep: list) -> sta_graph_desc:
    def a(x, dt):
        x = np.ascontiguousarray(x, dtype=dt)
        keep.append(x)
        return x.ctypes.data

    return sta_graph_desc(d.n_pins, d.n_cells, d.n_nets, d.n_pi, d.n_po, None, None, None, None, None,
                          a(d.net_driver, np.int32), a(d.net_sink_ptr, np.int32), a(d.net_sink_pin, np.int32),
                          STA_HOST)


def estimate_rc_backward(d, pin_x, pin_y, rc, r_x, r_y, c_x, c_y, grad_res, grad_cap, stream=None):
    """(dJ/dx, dJ/dy) per pin through the trees `rc` of estimate_rc, from
    dJ/dR and dJ/dC per node.  Host numpy arrays in and out, or cuda tensors
    in and out."""
    keep: list = []
    g = _net_graph(d, keep)
    w = sta_wire_params(r_x, r_y, c_x, c_y)
    if hasattr(pin_x, "data_ptr"):
        import torch
        dev = pin_x.device
        args = [t.contiguous() for t in (pin_x.float(), pin_y.float(), rc["parent"], rc["sink_node"],
                                         grad_res.float(), grad_cap.float())]
        gx = torch.empty(max(d.n_pins, 1), dtype=torch.float32, device=dev)
        gy = torch.empty(max(d.n_pins, 1), dtype=torch.float32, device=dev)
        sta_estimate_rc_backward(g, args[0], args[1], w, args[2], args[3], args[4], args[5], gx, gy, STA_DEVICE,
                                 stream if stream is not None else torch.cuda.current_stream(dev))
        return gx[: d.n_pins], gy[: d.n_pins]
    arrs = [np.ascontiguousarray(v, dt) for v, dt in ((pin_x, np.float32), (pin_y, np.float32),
                                                       (rc["parent"], np.int32), (rc["sink_node"], np.int32),
                                                       (grad_res, np.float32), (grad_cap, np.float32))]
    gx = np.zeros(d.n_pins, np.float32)
    gy = np.zeros(d.n_pins, np.float32)
    sta_estimate_rc_backward(g, *arrs[:2], w, *arrs[2:], gx, gy, STA_HOST, stream)
    return gx, gy


PHASES = ("rc_small", "rc_big", "forward", "backward", "reduce", "sort", "adjoint_sweep", "adjoint_rc")


# ------------------------------------------------------------------ owner

def descriptors(d, keep: list):
    """Host-memory descriptors for a synth.Design-shaped object.  Arrays that
    the descriptors point to are appended to `keep` (the caller holds them)."""

    def a(x, dt):
        x = np.ascontiguousarray(x, dtype=dt)
        keep.append(x)
        return x.ctypes.data

    g = sta_graph_desc(d.n_pins, d.n_cells, d.n_nets, d.n_pi, d.n_po,
                       a(d.pin_kind, np.int32), a(d.cell_type, np.int32), a(d.cell_in_ptr, np.int32),
                       a(d.cell_in_pin, np.int32), a(d.cell_out_pin, np.int32),
                       a(d.net_driver, np.int32), a(d.net_sink_ptr, np.int32),
                       a(d.net_sink_pin, np.int32), STA_HOST)
    rc = sta_rc_desc(int(d.n_nodes), a(d.net_node_ptr, np.int64), a(d.parent, np.int32),
                     a(d.res_kohm, np.float32), a(d.cap_ff, np.float32), a(d.sink_node, np.int32),
                     STA_HOST)
    lib = sta_lib_desc(d.n_types, d.nx, d.ny, a(d.n_inputs, np.int32), a(d.sense, np.int32),
                       a(d.pin_cap_ff, np.float32), a(d.slew_axis, np.float32),
                       a(d.load_axis, np.float32), a(d.tables, np.float32), float(d.po_cap_ff))
    cons = sta_constraints(a(d.pi_at, np.float32), a(d.pi_slew, np.float32), a(d.po_rat, np.float32),
                           (ctypes.c_float * 4)(*[float(v) for v in d.dangling_rat]))
    return g, rc, lib, cons


def _lib_key(d) -> bytes:
    """Identity of a design's library by content."""
    import hashlib
    h = hashlib.sha1()
    h.update(np.int32([d.n_types, d.nx, d.ny]).tobytes())
    for name in ("n_inputs", "sense", "pin_cap_ff", "slew_axis", "load_axis", "tables"):
        h.update(np.ascontiguousarray(getattr(d, name)).tobytes())
    h.update(np.float32(d.po_cap_ff).tobytes())
    return h.digest()


class STA:
    """One timing context on the current HIP device: of one design, or of a
    batch when given a list of designs that share one library."""

    def __init__(self, design, **opts):
        batch = isinstance(design, (list, tuple))
        designs = list(design) if batch else [design]
        o = sta_options_default()
        o.dangling_policy = int(designs[0].dangling_policy)
        for k, v in opts.items():
            setattr(o, k, v)
        keep: list = []
        descs = [descriptors(d, keep) for d in designs]
        if batch:
            # designs whose library arrays are equal share one library descriptor
            keys = [_lib_key(d) for d in designs]
            if all(k == keys[0] for k in keys):
                self.ctx = sta_batch_create([x[0] for x in descs], [x[1] for x in descs], descs[0][2],
                                            [x[3] for x in descs], o)
            else:
                first = {}
                libs = [descs[first.setdefault(k, i)][2] for i, k in enumerate(keys)]
                self.ctx = sta_batch_create_libs([x[0] for x in descs], [x[1] for x in descs], libs,
                                                 [x[3] for x in descs], o)
        else:
            g, rc, lib, cons = descs[0]
            self.ctx = sta_create(g, rc, lib, cons, o)
        self.n_designs = len(designs)
        self.info = sta_get_info(self.ctx)
        self.opts = o
        self._n_arcs = int(sum(int(d.cell_in_ptr[-1]) for d in designs))

    def close(self):
        if getattr(self, "ctx", None):
            sta_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def update(self, stream=None):
        sta_update_timing(self.ctx, stream)

    def update_incremental(self, nets, stream=None):
        """Incremental update after the caps of `nets` (caller net ids) changed."""
        mem = STA_DEVICE if hasattr(nets, "data_ptr") else STA_HOST
        sta_update_timing_incremental(self.ctx, nets, mem, stream)

    def set_wire_caps(self, cap, stream=None):
        mem = STA_DEVICE if hasattr(cap, "data_ptr") else STA_HOST
        sta_set_wire_caps(self.ctx, cap, mem, stream)

    def timing(self):
        n = self.info.n_pins
        at, slew, rat = (np.zeros((n, 4), np.float32) for _ in range(3))
        crit = np.zeros((n, 4), np.int8)
        sta_report_timing(self.ctx, at, slew, rat if self.opts.mode == 0 else None, crit)
        return {"at": at, "slew": slew, "rat": rat, "crit": crit}

    def slack(self):
        n, ne = self.info.n_pins, self.info.n_endpoints
        ps = np.zeros((n, 4), np.float32)
        es = np.zeros((max(ne, 1), 2), np.float32)
        eo = np.zeros((2, max(ne, 1)), np.int32)
        wns, tns = sta_report_slack(self.ctx, ps if self.opts.mode == 0 else None, es,
                                    eo if self.opts.sort_endpoints else None)
        return {"slack": ps, "ep_slack": es[:ne], "ep_order": eo[:, :ne], "wns": wns, "tns": tns}

    def levels(self):
        n = self.info.n_pins
        lv, lo = np.zeros(n, np.int32), np.zeros(n, np.int32)
        sta_report_levels(self.ctx, lv, lo)
        return lv, lo

    def rc(self):
        L = np.zeros(self.info.n_nets, np.float32)
        d = np.zeros(max(1, self.info.n_sinks), np.float32)
        q = np.zeros(max(1, self.info.n_sinks), np.float32)
        sta_report_rc(self.ctx, L, d, q)
        return L, d[: self.info.n_sinks], q[: self.info.n_sinks]

    def endpoints(self):
        e = np.zeros(max(1, self.info.n_endpoints), np.int32)
        sta_report_endpoints(self.ctx, e)
        return e[: self.info.n_endpoints]

    def paths(self, k, per_endpoint=1, slack_below=float("inf"), el=1):
        return sta_report_paths(self.ctx, k, per_endpoint, slack_below, el, self.info.n_levels)

    def batch_offsets(self):
        return sta_batch_offsets(self.ctx)

    def batch_report(self):
        return sta_batch_report(self.ctx, self.n_designs)

    def autotune(self, reps=5, stream=None):
        r = sta_autotune(self.ctx, reps, stream)
        self.opts.sched = r.sched
        self.opts.sweep_blocks = r.sweep_blocks
        self.opts.overlap = r.overlap
        return r

    def phase_times(self):
        return sta_get_phase_times(self.ctx)

    def backward(self, g_tns=1.0, g_wns=0.0):
        """Host gradients of g_tns*TNS_g + g_wns*WNS_g (smooth mode)."""
        gc = np.zeros(int(self.info.n_nodes), np.float32)
        gr = np.zeros(int(self.info.n_nodes), np.float32)
        gl = np.zeros(self.info.n_pins, np.float32)
        n_arcs = self._n_arcs
        ga = np.zeros((max(n_arcs, 1), 4), np.float32)
        sta_backward(self.ctx, g_tns, g_wns, gc, gr, gl, ga)
        return {"grad_wire_cap": gc, "grad_wire_res": gr, "grad_pin_load": gl, "grad_arc_delay": ga[:n_arcs]}


def _smooth_function():
    import torch

    class SmoothTiming(torch.autograd.Function):
        """(TNS_g, WNS_g) of the late views as a differentiable function of the RC
        node caps (caller node order, a float32 cuda tensor).  forward: caps ->
        sta_set_wire_caps + sta_update_timing on the current stream; backward:
        sta_backward writes d/d(caps) straight into a torch-owned buffer."""

        @staticmethod
        def forward(ctx, caps, timer):
            stream = torch.cuda.current_stream()
            caps = caps.contiguous()
            sta_set_wire_caps(timer.ctx, caps, STA_DEVICE, stream)
            sta_update_timing(timer.ctx, stream)
            wns, tns = sta_report_slack(timer.ctx, None, None, None, STA_HOST, stream)
            ctx.timer = timer
            ctx.n = caps.numel()
            return torch.tensor([tns[1], wns[1]], dtype=torch.float64, device=caps.device)

        @staticmethod
        def backward(ctx, grad_out):
            g = grad_out.detach().cpu()
            grad = torch.empty(ctx.n, dtype=torch.float32, device=grad_out.device)
            sta_backward(ctx.timer.ctx, float(g[0]), float(g[1]), grad, None, None, None, STA_DEVICE,
                         torch.cuda.current_stream())
            return grad, None

    return SmoothTiming


_SMOOTH = None


def smooth_timing(caps, timer):
    """Differentiable (TNS_g, WNS_g) of a smooth-mode STA context wrt node caps."""
    global _SMOOTH
    if _SMOOTH is None:
        _SMOOTH = _smooth_function()
    return _SMOOTH.apply(caps, timer)
