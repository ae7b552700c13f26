"""Seeded synthetic STA designs (netlist CSR, RC CSR, NLDM library, constraints).

The generator itself is C (``synth.c``, SplitMix64 streams); this module only
marshals its output into numpy arrays.  It holds none of the timing
arithmetic, so both the FP64 oracle and the GPU path may use it.

Named workloads follow the paper's scale range: the paper's designs span 66k to
4.2M pins (Table I) and up to 12M nets (Table IV); the tiny, 1M-pin and 10M-pin
designs below bracket that range.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libstasynth.so")


class _Cfg(ctypes.Structure):
    _fields_ = [
        ("n_cells", ctypes.c_int64),
        ("n_levels", ctypes.c_int32), ("n_pi", ctypes.c_int32), ("n_po", ctypes.c_int32),
        ("fanout_mu", ctypes.c_double),
        ("fanout_cap", ctypes.c_int32),
        ("n_types", ctypes.c_int32),
        ("n_heavy", ctypes.c_int32),
        ("heavy_frac", ctypes.c_double),
        ("n_hf", ctypes.c_int32), ("hf_min", ctypes.c_int32), ("hf_max", ctypes.c_int32),
        ("rat_ps", ctypes.c_double), ("rat_early_ps", ctypes.c_double),
        ("pi_at_ps", ctypes.c_double),
        ("pi_slew_ps", ctypes.c_double), ("po_cap_ff", ctypes.c_double),
        ("dangling_policy", ctypes.c_int32),
        ("shuffle", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("lib_seed", ctypes.c_uint64),
    ]


_P32 = ctypes.POINTER(ctypes.c_int32)
_P64 = ctypes.POINTER(ctypes.c_int64)
_PF = ctypes.POINTER(ctypes.c_float)


class _Design(ctypes.Structure):
    _fields_ = [
        ("n_pins", ctypes.c_int32), ("n_cells", ctypes.c_int32), ("n_nets", ctypes.c_int32),
        ("n_pi", ctypes.c_int32), ("n_po", ctypes.c_int32), ("n_sinks", ctypes.c_int32),
        ("n_cell_in", ctypes.c_int32),
        ("n_nodes", ctypes.c_int64),
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
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is not built; run __graft_entry__.build()")
        _lib = ctypes.CDLL(_LIB_PATH)
        _lib.synth_generate.restype = ctypes.POINTER(_Design)
        _lib.synth_generate.argtypes = [ctypes.POINTER(_Cfg)]
        _lib.synth_free.restype = None
        _lib.synth_free.argtypes = [ctypes.POINTER(_Design)]
    return _lib


@dataclass
class SynthConfig:
    n_cells: int
    n_levels: int
    n_pi: int
    n_po: int
    fanout_mu: float = 2.0
    fanout_cap: int = 8
    n_types: int = 8
    n_heavy: int = 0
    heavy_frac: float = 0.0
    n_hf: int = 0
    hf_min: int = 1000
    hf_max: int = 10000
    rat_ps: float = 500.0
    rat_early_ps: float = 500.0
    pi_at_ps: float = 0.0
    pi_slew_ps: float = 20.0
    po_cap_ff: float = 2.0
    dangling_policy: int = 0
    shuffle: int = 0
    seed: int = 1
    lib_seed: int = 0  # library tables / pin caps from this seed; 0 = seed


@dataclass
class Design:
    """Caller-format design: every array is in the layout the C ABI takes."""
    n_pins: int
    n_cells: int
    n_nets: int
    n_pi: int
    n_po: int
    n_sinks: int
    n_nodes: int
    pin_kind: np.ndarray
    cell_type: np.ndarray
    cell_in_ptr: np.ndarray
    cell_in_pin: np.ndarray
    cell_out_pin: np.ndarray
    net_driver: np.ndarray
    net_sink_ptr: np.ndarray
    net_sink_pin: np.ndarray
    net_node_ptr: np.ndarray
    parent: np.ndarray
    res_kohm: np.ndarray
    cap_ff: np.ndarray
    sink_node: np.ndarray
    n_types: int
    nx: int
    ny: int
    n_inputs: np.ndarray
    sense: np.ndarray
    pin_cap_ff: np.ndarray
    slew_axis: np.ndarray
    load_axis: np.ndarray
    tables: np.ndarray
    po_cap_ff: float
    pi_at: np.ndarray
    pi_slew: np.ndarray
    po_rat: np.ndarray
    dangling_rat: np.ndarray
    dangling_policy: int
    cfg: SynthConfig | None = None
    extra: dict = field(default_factory=dict)

    def copy(self) -> "Design":
        kw = {}
        for k, v in self.__dict__.items():
            kw[k] = v.copy() if isinstance(v, np.ndarray) else v
        return Design(**kw)


def _arr(ptr, n, dtype):
    if n == 0:
        return np.zeros(0, dtype=dtype)
    return np.ctypeslib.as_array(ptr, shape=(n,)).astype(dtype, copy=True)


def generate(cfg: SynthConfig) -> Design:
    lib = _load()
    c = _Cfg(cfg.n_cells, cfg.n_levels, cfg.n_pi, cfg.n_po, cfg.fanout_mu, cfg.fanout_cap,
             cfg.n_types, cfg.n_heavy, cfg.heavy_frac, cfg.n_hf, cfg.hf_min, cfg.hf_max,
             cfg.rat_ps, cfg.rat_early_ps, cfg.pi_at_ps, cfg.pi_slew_ps, cfg.po_cap_ff, cfg.dangling_policy,
             cfg.shuffle, cfg.seed, cfg.lib_seed)
    p = lib.synth_generate(ctypes.byref(c))
    if not p:
        raise ValueError(f"synth_generate rejected config {cfg}")
    d = p.contents
    try:
        T, NX, NY = d.n_types, d.nx, d.ny
        out = Design(
            n_pins=d.n_pins, n_cells=d.n_cells, n_nets=d.n_nets, n_pi=d.n_pi, n_po=d.n_po,
            n_sinks=d.n_sinks, n_nodes=d.n_nodes,
            pin_kind=_arr(d.pin_kind, d.n_pins, np.int32),
            cell_type=_arr(d.cell_type, d.n_cells, np.int32),
            cell_in_ptr=_arr(d.cell_in_ptr, d.n_cells + 1, np.int32),
            cell_in_pin=_arr(d.cell_in_pin, d.n_cell_in, np.int32),
            cell_out_pin=_arr(d.cell_out_pin, d.n_cells, np.int32),
            net_driver=_arr(d.net_driver, d.n_nets, np.int32),
            net_sink_ptr=_arr(d.net_sink_ptr, d.n_nets + 1, np.int32),
            net_sink_pin=_arr(d.net_sink_pin, d.n_sinks, np.int32),
            net_node_ptr=_arr(d.net_node_ptr, d.n_nets + 1, np.int64),
            parent=_arr(d.parent, d.n_nodes, np.int32),
            res_kohm=_arr(d.res_kohm, d.n_nodes, np.float32),
            cap_ff=_arr(d.cap_ff, d.n_nodes, np.float32),
            sink_node=_arr(d.sink_node, d.n_sinks, np.int32),
            n_types=T, nx=NX, ny=NY,
            n_inputs=_arr(d.n_inputs, T, np.int32),
            sense=_arr(d.sense, T, np.int32),
            pin_cap_ff=_arr(d.pin_cap_ff, T, np.float32),
            slew_axis=_arr(d.slew_axis, T * NX, np.float32).reshape(T, NX),
            load_axis=_arr(d.load_axis, T * NY, np.float32).reshape(T, NY),
            tables=_arr(d.tables, T * 4 * NX * NY, np.float32).reshape(T, 4, NX, NY),
            po_cap_ff=float(d.po_cap_ff),
            pi_at=_arr(d.pi_at, d.n_pi * 4, np.float32).reshape(d.n_pi, 4),
            pi_slew=_arr(d.pi_slew, d.n_pi * 4, np.float32).reshape(d.n_pi, 4),
            po_rat=_arr(d.po_rat, d.n_po * 4, np.float32).reshape(d.n_po, 4),
            dangling_rat=np.array(list(d.dangling_rat), dtype=np.float32),
            dangling_policy=int(d.dangling_policy),
            cfg=cfg,
        )
    finally:
        lib.synth_free(p)
    return out


# ---------------------------------------------------------------- workloads

def tiny_config(seed: int = 1, **kw) -> SynthConfig:
    """2,000 cells, 20 levels, 64 PI / 64 PO, fanout geometric mean 2 capped at 8,
    8 cell types, PI AT 0 / slew 20 ps, endpoint RAT 500 ps in all four views."""
    c = SynthConfig(n_cells=2000, n_levels=20, n_pi=64, n_po=64, fanout_mu=2.0, fanout_cap=8,
                    n_types=8, rat_ps=500.0, rat_early_ps=500.0, dangling_policy=0, seed=seed)
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def mid_config(seed: int = 2, n_cells: int = 400_000, n_levels: int = 60, **kw) -> SynthConfig:
    """1M-pin class: 400k cells, 60 uniform levels, 32 types, fanout mean 3 capped
    at 32, PI = PO = ceil(cells / levels), zero-fanout cell outputs are endpoints.
    Late endpoint RAT is 75 ps per level, which leaves a mix of violating and
    passing endpoints; early (hold-style) RAT is 50 ps."""
    npio = int(math.ceil(n_cells / n_levels))
    c = SynthConfig(n_cells=n_cells, n_levels=n_levels, n_pi=npio, n_po=npio, fanout_mu=3.0,
                    fanout_cap=32, n_types=32, rat_ps=75.0 * n_levels, rat_early_ps=50.0,
                    dangling_policy=1, seed=seed)
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def large_config(seed: int = 3, n_cells: int = 4_000_000, n_levels: int = 120, **kw) -> SynthConfig:
    """10M-pin class: 4M cells, 120 levels of which 4 (drawn from 2..120) hold 5% of
    the cells each, fanout mean 3 capped at 32, plus 20 high-fanout nets
    (log-uniform 1k..10k sinks, about 1% of all sinks) driven by PIs or level-1
    cells.  PI = PO = ceil(cells / levels)."""
    npio = int(math.ceil(n_cells / n_levels))
    c = SynthConfig(n_cells=n_cells, n_levels=n_levels, n_pi=npio, n_po=npio, fanout_mu=3.0,
                    fanout_cap=32, n_types=32, n_heavy=4, heavy_frac=0.05, n_hf=20,
                    hf_min=1000, hf_max=10000, rat_ps=75.0 * n_levels, rat_early_ps=50.0,
                    dangling_policy=1,
                    seed=seed)
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def batch_configs(n_designs: int = 256, base_seed: int = 5_000_000,
                  min_cells: int = 1000, max_cells: int = 200_000) -> list[SynthConfig]:
    """Uneven batch: per design, cells log-uniform in [min_cells, max_cells] and
    levels uniform in 10..80, drawn from the design's own seed; otherwise the
    1M-pin generator settings.  All designs of a batch share one cell library
    (one technology), drawn from the first design's seed."""
    out = []
    for i in range(n_designs):
        seed = base_seed + i
        rng = np.random.Generator(np.random.PCG64(seed))
        cells = int(round(math.exp(rng.uniform(math.log(min_cells), math.log(max_cells)))))
        levels = int(rng.integers(10, 81))
        levels = min(levels, cells)
        out.append(mid_config(seed=seed, n_cells=cells, n_levels=levels, lib_seed=base_seed))
    return out


def corner_configs(base: SynthConfig, lib_seeds=(11, 12, 13, 14)) -> list[SynthConfig]:
    """The same netlist (base's seed and sizes) under one library per entry of
    lib_seeds, as a batch of corners: the library streams are independent of
    the netlist streams, so only the tables and pin caps differ."""
    return [dataclasses.replace(base, lib_seed=int(ls)) for ls in lib_seeds]


def mixed_batch_configs(n_designs: int = 256, n_libs: int = 4, base_seed: int = 5_000_000,
                        min_cells: int = 1000, max_cells: int = 200_000) -> list[SynthConfig]:
    """batch_configs with a library per design: design i takes library
    i mod n_libs (seeds base_seed + 1_000_000 + j), e.g. designs of several
    technologies or corners in one batch."""
    out = batch_configs(n_designs, base_seed, min_cells, max_cells)
    return [dataclasses.replace(c, lib_seed=base_seed + 1_000_000 + i % n_libs) for i, c in enumerate(out)]


def stats(d: Design) -> dict:
    """Realized size statistics of a generated design."""
    fo = np.diff(d.net_sink_ptr)
    nodes = np.diff(d.net_node_ptr)
    return {
        "pins": d.n_pins, "cells": d.n_cells, "nets": d.n_nets, "sinks": d.n_sinks,
        "rc_nodes": int(d.n_nodes), "cell_arcs": int(d.cell_in_ptr[-1]),
        "pi": d.n_pi, "po": d.n_po,
        "fanout_mean": float(fo.mean()), "fanout_max": int(fo.max()),
        "zero_fanout_drivers": int((fo == 0).sum()),
        "nodes_per_net_max": int(nodes.max()),
        "nodes_per_sink": float((d.n_nodes - d.n_nets) / max(1, d.n_sinks)),
    }


def place(d: Design, seed: int = 1, sigma_um: float = 6.0, cell_pitch_um: float = 2.0):
    """Synthetic placement (pin positions for RC estimation): PIs uniform on a
    square die of side cell_pitch_um * sqrt(cells + PIs); each cell at the
    position of the driver of its first input plus a seeded Gaussian offset
    (sigma_um per axis), clamped to the die; every pin at its cell's position,
    a PO at its driver's.  Nets are then mostly local, with the wire lengths a
    placer leaves.  Returns float32 (x, y) in micrometres per caller pin."""
    rng = np.random.default_rng(seed)
    side = float(cell_pitch_um * np.sqrt(d.n_cells + d.n_pi))
    x = np.full(d.n_pins, np.nan, np.float64)
    y = np.full(d.n_pins, np.nan, np.float64)
    kind = np.asarray(d.pin_kind)
    pis = np.flatnonzero(kind == 0)
    x[pis] = rng.uniform(0.0, side, pis.size)
    y[pis] = rng.uniform(0.0, side, pis.size)
    # driver pin of every sink pin
    nsp = np.asarray(d.net_sink_ptr)
    drv_of = np.full(d.n_pins, -1, np.int64)
    drv_of[np.asarray(d.net_sink_pin)] = np.repeat(np.asarray(d.net_driver), np.diff(nsp))
    first_in = np.asarray(d.cell_in_pin)[np.asarray(d.cell_in_ptr)[:-1]]
    src = drv_of[first_in]  # pin whose position a cell copies
    out = np.asarray(d.cell_out_pin)
    ox = rng.normal(0.0, sigma_um, d.n_cells)
    oy = rng.normal(0.0, sigma_um, d.n_cells)
    todo = np.ones(d.n_cells, bool)
    while todo.any():  # cells whose first input's driver is placed, level by level
        ready = todo & ~np.isnan(x[src])
        if not ready.any():
            raise ValueError("placement: unplaced drivers (cycle?)")
        c = np.flatnonzero(ready)
        x[out[c]] = np.clip(x[src[c]] + ox[c], 0.0, side)
        y[out[c]] = np.clip(y[src[c]] + oy[c], 0.0, side)
        todo[c] = False
    cell_of_in = np.repeat(np.arange(d.n_cells), np.diff(np.asarray(d.cell_in_ptr)))
    cin = np.asarray(d.cell_in_pin)
    x[cin] = x[out[cell_of_in]]
    y[cin] = y[out[cell_of_in]]
    pos = np.flatnonzero(kind == 3)
    x[pos] = x[drv_of[pos]]
    y[pos] = y[drv_of[pos]]
    return x.astype(np.float32), y.astype(np.float32)


def with_rc(d: Design, rc: dict) -> Design:
    """A copy of d with its RC trees replaced (an RC-CSR dict as returned by
    the RC estimation)."""
    e = d.copy()
    e.net_node_ptr = np.asarray(rc["net_node_ptr"], np.int64).copy()
    e.parent = np.asarray(rc["parent"], np.int32).copy()
    e.res_kohm = np.asarray(rc["res_kohm"], np.float32).copy()
    e.cap_ff = np.asarray(rc["cap_ff"], np.float32).copy()
    e.sink_node = np.asarray(rc["sink_node"], np.int32).copy()
    e.n_nodes = int(e.net_node_ptr[-1])
    return e
