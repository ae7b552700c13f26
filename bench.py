"""Timing-graph pins/s of one full static-timing update (RC pass, forward
AT/slew sweep, backward RAT/slack sweep, WNS/TNS, endpoint order) on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload 10M|1M|tiny] [--sched auto|0|1|2]

Prints ONE JSON line.  A step is one sta_update_timing over the whole design
with every input resident in HBM.  `roofline` prices the dominant kernel's
algorithmic bytes (each array element moved once per update) against 8 TB/s;
`cpu_baseline` times the FP64 oracle single-threaded on the same design.
Three side measurements ride along: `incremental` (sta_update_timing_incremental
after k random nets of the same design were re-capped), `adjoint` (smooth-mode
reverse pass time over smooth forward time on the 1M-pin design) and `batched`
(256 uneven designs timed as one batch against the sum of the same designs
timed one after another on one stream, each context tuned for itself).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "timing-graph pins/s (fwd+bwd STA) + % HBM peak; adjoint/forward time ratio"


def algorithmic_bytes(info, n_arcs: int) -> dict:
    """Compulsory HBM bytes per update, per kernel (each element moved once).
    Sizes: N_p pins, N_s sinks, N_n nets, N_c cells, N_a cell arcs, N_r RC
    nodes, N_po endpoints, V = 4 views."""
    Np, Ns, Nn, Nc = info.n_pins, info.n_sinks, info.n_nets, info.n_cells
    Nr, Na, Npo, V = info.n_nodes, n_arcs, info.n_endpoints, 4
    rc = 8 * (Nr - Nn) + 4 * Nr + 4 * Nn + 4 * Ns + 8 * Ns + 4 * Nn
    fwd = 4 * Np + 4 * (Ns + Na) + 8 * V * Np + 8 * Ns + 4 * Nn + 4 * Nc + 8 * V * Np + 4 * Nc
    bwd = 4 * Np + 4 * (Ns + Na) + 4 * V * Np + 4 * V * Na + 4 * Ns + 3 * 4 * V * Np + 4 * V * Npo
    return {"rc": rc, "forward": fwd, "backward": bwd, "total": rc + fwd + bwd}


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("paper_2511_11660_amd/csrc/sta_kernels.hip", "paper_2511_11660_amd/csrc/sta_internal.h"):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(sweep: str, workload: str):
    """HBM bytes of one sweep per update (summed over its launches) from the
    committed rocprofv3 FETCH_SIZE/WRITE_SIZE counters, scaled by the same
    counters on a plain device copy; None unless they were taken on the
    current kernel source."""
    path = os.path.join(ROOT, "profiles", f"traffic_{sweep}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    return t.get("bytes_per_update")


def host_cpu() -> dict:
    """CPU model and the hardware threads this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 0
    return {"cpu_model": model, "host_threads": n}


def cpu_baseline(design, n_pins: int, runs: int = 3) -> dict:
    """The FP64 oracle (plain C, one thread) on the whole design, median of
    `runs` updates.  Each is timed inside the oracle around what one
    sta_update_timing does (RC, forward, backward, slacks, WNS/TNS, endpoint
    order); the levelization and pin-role maps, which the GPU path builds once
    at create, and the Python-side array copies are outside the timed part."""
    import oracle
    ts = [oracle.sta(design)["update_seconds"] for _ in range(runs)]
    dt = sorted(ts)[len(ts) // 2]
    return {"value": n_pins / dt, "unit": "pins/s", "cores": 1, "kind": "oracle",
            "sample": f"{runs} FP64 updates of the same design ({n_pins} pins), RC through endpoint order "
                      f"timed inside the oracle, single thread, median {dt:.2f} s",
            **host_cpu()}


def _time_updates(ctxs, stream, steps):
    """Mean ms of `steps` rounds of one update on each context in ctxs,
    back to back on one stream."""
    import torch
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(steps):
        for c in ctxs:
            c.update(stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / steps


def adjoint_ratio(steps: int, sched: str = "auto") -> dict:
    """Smooth-mode update (LSE arrival merges, smooth TNS/WNS) and its reverse
    pass (sta_backward into device gradient buffers) on the 1M-pin design; the
    forward's schedule autotuned, or the one given."""
    import torch
    from paper_2511_11660_amd import synth
    from paper_2511_11660_amd.sta import STA
    d = synth.generate(synth.mid_config())
    s = STA(d, mode=1, gamma_ps=5.0, sort_endpoints=0, device=0, sched=0 if sched == "auto" else int(sched))
    if sched == "auto":
        chosen = s.autotune(reps=3).sched
    else:
        chosen = int(sched)
    stream = torch.cuda.current_stream()
    gc = torch.empty(int(d.n_nodes), dtype=torch.float32, device="cuda")
    gr = torch.empty(int(d.n_nodes), dtype=torch.float32, device="cuda")
    gl = torch.empty(d.n_pins, dtype=torch.float32, device="cuda")
    ga = torch.empty((int(d.cell_in_ptr[-1]), 4), dtype=torch.float32, device="cuda")
    from paper_2511_11660_amd.sta import STA_DEVICE, sta_backward
    for _ in range(3):
        s.update(stream)
        sta_backward(s.ctx, 1.0, 0.0, gc, gr, gl, ga, STA_DEVICE, stream)
    t_fwd = _time_updates([s], stream, steps)
    s.update(stream)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(steps):
        sta_backward(s.ctx, 1.0, 0.0, gc, gr, gl, ga, STA_DEVICE, stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    t_bwd = ev0.elapsed_time(ev1) / steps
    s.close()
    return {"workload": "1M-pin synthetic design, smooth mode gamma 5 ps", "pins": d.n_pins,
            "schedule": _SCHED_NAMES[chosen], "forward_ms": t_fwd, "backward_ms": t_bwd,
            "ratio": t_bwd / t_fwd}


def batched_vs_per_design(steps: int, n_designs: int, n_libs: int = 1) -> dict:
    """The uneven batch timed as one union against the same designs one by
    one; with n_libs > 1 design i takes library i mod n_libs (per-design
    libraries, e.g. several technologies or corners in one batch)."""
    import torch
    from paper_2511_11660_amd import synth
    from paper_2511_11660_amd.sta import STA
    cfgs = synth.batch_configs(n_designs) if n_libs <= 1 else synth.mixed_batch_configs(n_designs, n_libs)
    designs = [synth.generate(c) for c in cfgs]
    pins = sum(d.n_pins for d in designs)
    print(f"[bench] batch: {n_designs} designs, {pins} pins", file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream()
    b = STA(designs, device=0)
    rb = b.autotune(reps=3)
    t_batch = _time_updates([b], stream, steps)
    b.close()
    singles = []
    for d in designs:
        s = STA(d, device=0)
        s.autotune(reps=1)
        singles.append(s)
    t_seq = _time_updates(singles, stream, max(1, steps // 4))
    for s in singles:
        s.close()
    lib_note = "shared library" if n_libs <= 1 else f"design i with library i mod {n_libs}"
    return {"workload": f"{n_designs} uneven synthetic designs (1k-200k cells, 10-80 levels), {lib_note}",
            "libraries": max(1, n_libs),
            "designs": n_designs, "pins": pins, "schedule": _SCHED_NAMES[rb.sched],
            "batched_ms": t_batch, "per_design_sum_ms": t_seq, "speedup": t_seq / t_batch,
            "batched_pins_per_s": pins / (t_batch * 1e-3)}


def incremental_updates(design, sched: int, blocks: int, full_ms: float, sizes=(1, 100, 10000), reps: int = 3) -> dict:
    """sta_update_timing_incremental after the caps of k random nets changed
    (x1.5 or /1.5 on every node of each), median of `reps` calls per k, timed
    with events around the call (its host work included)."""
    import numpy as np
    import torch
    from paper_2511_11660_amd.sta import STA
    s = STA(design, sched=sched, sweep_blocks=blocks, device=0)
    stream = torch.cuda.current_stream()
    caps = design.cap_ff.astype(np.float32).copy()
    nnp = np.asarray(design.net_node_ptr)
    rng = np.random.default_rng(11)
    s.update(stream)
    s.update_incremental(np.zeros(0, np.int32), stream)  # allocations of the first call
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # the reference: one full update timed the same way (events around a
    # single call from an idle stream, its launch latency included)
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        ev0.record(stream)
        s.update(stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        ts.append(ev0.elapsed_time(ev1))
    out = {"workload": "10M-pin design, k random nets re-capped", "full_ms": full_ms,
           "full_single_call_ms": sorted(ts)[len(ts) // 2], "ms": {}}
    for k in sizes:
        ts = []
        for rep in range(reps):
            nets = rng.choice(design.n_nets, k, replace=False).astype(np.int32)
            f = np.float32(1.5 if rep % 2 == 0 else 1 / 1.5)
            for n in nets:
                caps[nnp[n]:nnp[n + 1]] *= f
            s.set_wire_caps(caps, stream)
            torch.cuda.synchronize()
            ev0.record(stream)
            s.update_incremental(nets, stream)
            ev1.record(stream)
            torch.cuda.synchronize()
            ts.append(ev0.elapsed_time(ev1))
        out["ms"][str(k)] = sorted(ts)[len(ts) // 2]
    s.close()
    return out


def rc_estimate_side(design, reps: int = 5) -> dict:
    """sta_estimate_rc on the whole design with every input and output in HBM
    (synthetic placement), median of `reps` calls timed with events around
    the call (its two host waits included)."""
    import numpy as np
    import torch
    from paper_2511_11660_amd import synth
    from paper_2511_11660_amd.sta import STA_DEVICE, sta_estimate_rc, sta_graph_desc, sta_wire_params
    x, y = synth.place(design, seed=1)
    dev = {k: torch.from_numpy(np.ascontiguousarray(getattr(design, k), np.int32)).cuda()
           for k in ("net_driver", "net_sink_ptr", "net_sink_pin")}
    dx, dy = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    g = sta_graph_desc(design.n_pins, design.n_cells, design.n_nets, design.n_pi, design.n_po, None, None, None,
                       None, None, dev["net_driver"].data_ptr(), dev["net_sink_ptr"].data_ptr(),
                       dev["net_sink_pin"].data_ptr(), STA_DEVICE)
    nn, ns = design.n_nets, int(design.net_sink_ptr[-1])
    nodes = nn + 3 * ns
    ptr = torch.empty(nn + 1, dtype=torch.int64, device="cuda")
    par = torch.empty(nodes, dtype=torch.int32, device="cuda")
    res = torch.empty(nodes, dtype=torch.float32, device="cuda")
    cap = torch.empty(nodes, dtype=torch.float32, device="cuda")
    sink = torch.empty(ns, dtype=torch.int32, device="cuda")
    w = sta_wire_params(0.002, 0.002, 0.2, 0.2)
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ts = []
    for _ in range(reps + 1):
        torch.cuda.synchronize()
        ev0.record(stream)
        sta_estimate_rc(g, dx, dy, w, ptr, par, res, cap, sink, STA_DEVICE, stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        ts.append(ev0.elapsed_time(ev1))
    ms = sorted(ts[1:])[reps // 2]
    # the gradient to positions through the same trees, from random node gradients
    from paper_2511_11660_amd.sta import sta_estimate_rc_backward
    gen = torch.Generator(device="cuda").manual_seed(3)
    g_res = torch.rand(nodes, device="cuda", generator=gen) - 0.5
    g_cap = torch.rand(nodes, device="cuda", generator=gen) - 0.5
    gx = torch.empty(design.n_pins, dtype=torch.float32, device="cuda")
    gy = torch.empty_like(gx)
    tb = []
    for _ in range(reps + 1):
        torch.cuda.synchronize()
        ev0.record(stream)
        sta_estimate_rc_backward(g, dx, dy, w, par, sink, g_res, g_cap, gx, gy, STA_DEVICE, stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        tb.append(ev0.elapsed_time(ev1))
    ms_b = sorted(tb[1:])[reps // 2]
    # net CSR and driver (12 B/net), sink pins (4 B/sink), positions of every
    # net pin (8 B), outputs: node_ptr 8 B/net, 12 B/node, sink_node 4 B/sink
    algo = 12 * nn + 4 * ns + 8 * (nn + ns) + 8 * nn + 12 * nodes + 4 * ns
    # wire length of the Steiner trees against the rectilinear minimum spanning
    # tree, over 2000 sampled nets of at least 3 pins (r_x = r_y, so the length
    # is the sum of R over r)
    from scipy.sparse.csgraph import minimum_spanning_tree
    res_h, ptr_h = res.cpu().numpy().astype(np.float64), ptr.cpu().numpy()
    nsp = np.asarray(design.net_sink_ptr, np.int64)
    cand = np.flatnonzero(np.diff(nsp) >= 2)
    steiner = mst = 0.0
    for n in np.random.default_rng(5).choice(cand, min(2000, cand.size), replace=False):
        pins = np.concatenate([[design.net_driver[n]], design.net_sink_pin[nsp[n]:nsp[n + 1]]])
        pts = np.unique(np.stack([x[pins], y[pins]], 1).astype(np.float64), axis=0)
        dm = np.abs(pts[:, None, :] - pts[None, :, :]).sum(-1)
        mst += float(minimum_spanning_tree(dm).toarray().sum())
        steiner += float(res_h[ptr_h[n]:ptr_h[n + 1]].sum()) / w.r_x
    return {"workload": "10M-pin design, synthetic placement, all arrays in HBM", "nets": nn, "sinks": ns,
            "max_fanout": int(np.diff(design.net_sink_ptr).max()), "ms": ms,
            "pins_per_s": (nn + ns) / (ms * 1e-3), "algorithmic_GBps": algo / (ms * 1e-3) / 1e9,
            "backward_ms": ms_b, "tree": "rectilinear Steiner (shortest-path joins)",
            "wirelength_over_spanning_tree": steiner / mst}


def reduced_order_side(design, sched: int, blocks: int, steps: int, full_ms: float) -> dict:
    """Full updates of the same design with the reduced-order (Arnoldi) net
    delays instead of Elmore, on the schedule the context tunes for itself
    (as the adjoint and batched measurements do)."""
    import torch
    from paper_2511_11660_amd.sta import STA
    s = STA(design, sched=sched, sweep_blocks=blocks, delay_model=1, device=0)
    stream = torch.cuda.current_stream()
    r = s.autotune(reps=3, stream=stream)
    s.update(stream)
    ms = _time_updates([s], stream, steps)
    s.close()
    return {"workload": "10M-pin design, reduced-order net delays", "schedule": _SCHED_NAMES[r.sched], "ms": ms,
            "elmore_ms": full_ms, "pins_per_s": design.n_pins / (ms * 1e-3)}


def paths_side(design, sched: int, blocks: int, reps: int = 5) -> dict:
    """sta_report_paths after one full update of the same design: the k worst
    late paths (at most per_endpoint per endpoint) into device arrays, median
    of `reps` calls timed with events around the call (its host waits
    included)."""
    import ctypes

    import torch
    from paper_2511_11660_amd.sta import STA, STA_DEVICE, load, sta_path_query
    s = STA(design, sched=sched, sweep_blocks=blocks, device=0)
    stream = torch.cuda.current_stream()
    s.update(stream)
    k, per_ep = 10000, 4
    lmax = s.info.n_levels
    dev = dict(device="cuda")
    ptr = torch.empty(k + 1, dtype=torch.int32, **dev)
    pins = torch.empty(k * lmax, dtype=torch.int32, **dev)
    rf = torch.empty(k * lmax, dtype=torch.int8, **dev)
    slack = torch.empty(k, dtype=torch.float32, **dev)
    ep = torch.empty(k, dtype=torch.int32, **dev)
    q = sta_path_query(k, per_ep, float("inf"), 1)
    n = ctypes.c_int32(0)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ts = []
    for _ in range(reps + 1):
        torch.cuda.synchronize()
        ev0.record(stream)
        rc = load().sta_report_paths(s.ctx, ctypes.byref(q), ctypes.byref(n), ptr.data_ptr(), pins.data_ptr(),
                                     rf.data_ptr(), slack.data_ptr(), ep.data_ptr(), STA_DEVICE, stream.cuda_stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        if rc != 0:
            raise RuntimeError(f"sta_report_paths failed: {rc}")
        ts.append(ev0.elapsed_time(ev1))
    n_pin_total = int(ptr[n.value].item()) if n.value > 0 else 0
    s.close()
    ms = sorted(ts[1:])[reps // 2]
    return {"workload": "10M-pin design after a full update, worst late paths", "k": k, "per_endpoint": per_ep,
            "paths": n.value, "path_pins": n_pin_total, "ms": ms, "paths_per_s": n.value / (ms * 1e-3)}


_SCHED_NAMES = {0: "persistent", 1: "per-level", 2: "graph", 3: "dataflow"}


def copy_calibration(mib: int, reps: int) -> int:
    """A plain device copy of known size, so HBM counters (FETCH_SIZE,
    WRITE_SIZE) can be scaled: each launch reads and writes mib MiB."""
    import torch
    n = mib * 1024 * 1024 // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        b.copy_(a)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    print(json.dumps({"copy_mib": mib, "ms": ms, "GBps_read_plus_write": 2 * mib * 1048576 / (ms * 1e-3) / 1e9}))
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="10M", choices=["10M", "1M", "tiny"])
    ap.add_argument("--sched", default="auto",
                    help="auto (tuned at setup), 0 persistent, 1 one launch per level, 2 HIP graph, 3 dataflow")
    ap.add_argument("--overlap", type=int, default=1, choices=[0, 1],
                    help="with --sched 1 or 2: side-stream phases on (1) or off (0); auto tunes it")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-side", action="store_true", help="skip every side measurement")
    ap.add_argument("--side", default="incremental,rc_estimate,reduced_order,adjoint,batched,batched_libs,paths",
                    help="comma list of side measurements to run")
    ap.add_argument("--batch-designs", type=int, default=256)
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB (counter calibration)")
    args = ap.parse_args()
    if args.copy_calib:
        return copy_calibration(args.copy_calib, args.steps)
    if args.gpus != 1:
        print(json.dumps({"error": "the timer runs on one GPU; splitting a design over several GPUs "
                                   "is not implemented", "n_gpus": args.gpus}))
        return 2

    import numpy as np
    import torch

    from paper_2511_11660_amd import synth
    from paper_2511_11660_amd.sta import PHASES, STA

    torch.cuda.set_device(0)
    cfg = {"10M": synth.large_config, "1M": synth.mid_config, "tiny": synth.tiny_config}[args.workload]()
    t0 = time.perf_counter()
    design = synth.generate(cfg)
    t_gen = time.perf_counter() - t0
    print(f"[bench] generated {design.n_pins} pins in {t_gen:.1f}s", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    s = STA(design, sched=0 if args.sched == "auto" else int(args.sched), overlap=args.overlap, device=0)
    t_create = time.perf_counter() - t0
    info = s.info
    print(f"[bench] created context in {t_create:.1f}s: {info.n_cell_levels} cell levels, "
          f"{info.n_endpoints} endpoints, {info.n_big_nets} big nets", file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream()
    tuned = None
    if args.sched == "auto":
        tuned = s.autotune(reps=5, stream=stream)
        print(f"[bench] autotune: {_SCHED_NAMES[tuned.sched]} grid {tuned.sweep_blocks} overlap {tuned.overlap} "
              f"({tuned.ms:.3f} ms, {tuned.n_tried} candidates)", file=sys.stderr, flush=True)
    sched, s_blocks = s.opts.sched, s.opts.sweep_blocks
    for _ in range(args.warmup):
        s.update(stream)
    torch.cuda.synchronize()

    # timed region: K back-to-back updates on one stream
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        s.update(stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    print(f"[bench] {ms:.3f} ms per update", file=sys.stderr, flush=True)

    wns_tns = s.slack()
    s.close()
    # per-kernel durations: the library's HIP events on the same stream (a
    # graph replay is not separable into phases, so its kernels are timed in
    # the per-level launch sequence the graph holds)
    prof = STA(design, sched=1 if sched == 2 else sched, sweep_blocks=s_blocks, profile=1, device=0)
    for _ in range(args.warmup):
        prof.update(stream)
    phase = np.zeros(len(PHASES))
    for _ in range(args.steps):
        prof.update(stream)
        phase += prof.phase_times()
    phase /= args.steps
    prof.close()

    # the second denominator: a plain vector copy kernel of the library, 1 GiB
    from paper_2511_11660_amd.sta import sta_measure_copy
    cbuf = torch.empty(2 << 30, dtype=torch.uint8, device="cuda")
    copy_ms = sta_measure_copy(cbuf[: 1 << 30], cbuf[1 << 30:], 1 << 30, 10, stream)
    copy_gbps = 2 * (1 << 30) / (copy_ms * 1e-3) / 1e9
    del cbuf

    # the latency floor of a level-synchronous sweep at this design's shape:
    # one launch per level, each an index load, a 32-byte gather over the sink
    # states and a 32-byte store for every sink of an average level
    from paper_2511_11660_amd.sta import sta_measure_level_floor
    n_lv = info.n_cell_levels + 1
    floor_ms = sta_measure_level_floor(n_lv, max(1, info.n_sinks // n_lv), info.n_sinks, 5, stream)

    n_arcs = int(design.cell_in_ptr[-1])
    ab = algorithmic_bytes(info, n_arcs)
    kern = {"forward": phase[PHASES.index("forward")], "backward": phase[PHASES.index("backward")],
            "rc": phase[PHASES.index("rc_small")] + phase[PHASES.index("rc_big")]}
    dom = max(kern, key=kern.get)
    achieved = ab[dom] / (kern[dom] * 1e-3) / 1e9
    traffic = measured_traffic(dom, args.workload)
    out = {
        "metric": METRIC,
        "value": info.n_pins / (ms * 1e-3),
        "unit": "pins/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded generator standing in for the paper's benchmark suites)",
        "config": {"workload": f"{args.workload}-pin synthetic STA design", "pins": info.n_pins,
                   "cells": info.n_cells, "nets": info.n_nets, "rc_nodes": int(info.n_nodes),
                   "cell_levels": info.n_cell_levels, "endpoints": info.n_endpoints,
                   "views": 4, "schedule": _SCHED_NAMES[sched], "overlap": int(s.opts.overlap)},
        "hbm_frac_whole_update": ab["total"] / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "level_floor": {"ms_per_sweep": floor_ms, "levels": n_lv, "items_per_level": max(1, info.n_sinks // n_lv),
                        "forward_over_floor": kern["forward"] / floor_ms,
                        "backward_over_floor": kern["backward"] / floor_ms},
        "phase_ms": {k: float(v) for k, v in zip(PHASES, phase)},
        "roofline": {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "algorithmic_bytes": ab[dom],
                     "copy_GBps": copy_gbps, "frac_of_copy": achieved / copy_gbps},
        "wns_ps": [float(x) for x in wns_tns["wns"]],
        "tns_ps": [float(x) for x in wns_tns["tns"]],
    }
    side = set() if args.no_side else set(args.side.split(","))
    if "incremental" in side:
        print("[bench] incremental updates", file=sys.stderr, flush=True)
        out["incremental"] = incremental_updates(design, sched, s_blocks, ms)
    if "rc_estimate" in side:
        print("[bench] RC estimation from pin positions", file=sys.stderr, flush=True)
        out["rc_estimate"] = rc_estimate_side(design)
    if "reduced_order" in side:
        print("[bench] reduced-order delays", file=sys.stderr, flush=True)
        out["reduced_order"] = reduced_order_side(design, sched, s_blocks, args.steps, ms)
    if "adjoint" in side:
        print("[bench] adjoint ratio (1M-pin smooth)", file=sys.stderr, flush=True)
        out["adjoint"] = adjoint_ratio(args.steps, args.sched)
    if "paths" in side:
        print("[bench] top-k path report", file=sys.stderr, flush=True)
        out["paths"] = paths_side(design, sched, s_blocks)
    if "batched" in side:
        print("[bench] batched vs per-design", file=sys.stderr, flush=True)
        out["batched"] = batched_vs_per_design(args.steps, args.batch_designs)
    if "batched_libs" in side:
        print("[bench] batched with per-design libraries vs per-design", file=sys.stderr, flush=True)
        out["batched_libs"] = batched_vs_per_design(args.steps, args.batch_designs, n_libs=4)
    if not args.no_cpu_baseline:
        print("[bench] timing the FP64 oracle on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(design, info.n_pins)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
