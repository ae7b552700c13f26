"""Batched form on the GPU: several designs (sharing one library, or each
with its own: corners) timed as one union graph.  Each design's slice of the batched results is compared bit for
bit with the same design timed alone (same kernels, same per-pin arithmetic
order, same reduction partition), and against the FP64 oracle per design."""
import numpy as np
import pytest

import oracle
from paper_2511_11660_amd import synth
from paper_2511_11660_amd.sta import (STA, STA_SCHED_FLOW, STA_SCHED_GRAPH, STA_SCHED_PER_LEVEL,
                                      STA_SCHED_PERSISTENT)
from parity import compare_full, run_gpu

pytestmark = pytest.mark.gpu


def _designs(n, base_seed, min_cells, max_cells):
    cfgs = synth.batch_configs(n, base_seed=base_seed, min_cells=min_cells, max_cells=max_cells)
    return [synth.generate(c) for c in cfgs]


def split(designs, gpu, offsets, wns, tns):
    """Per-design views of a batched run (the run_gpu dict of the union)."""
    pin_off, ep_off, _ = offsets
    out = []
    net_off = np.concatenate([[0], np.cumsum([d.n_nets for d in designs])])
    sink_off = np.concatenate([[0], np.cumsum([d.n_sinks for d in designs])])
    lv, lo = gpu["levels"]
    L, dd, q = gpu["rc"]
    t, s = gpu["timing"], gpu["slack"]
    for i, d in enumerate(designs):
        p0, p1 = int(pin_off[i]), int(pin_off[i + 1])
        e0, e1 = int(ep_off[i]), int(ep_off[i + 1])
        n0, n1 = int(net_off[i]), int(net_off[i + 1])
        s0, s1 = int(sink_off[i]), int(sink_off[i + 1])
        mine = lo[(lo >= p0) & (lo < p1)] - p0
        out.append({
            "levels": (lv[p0:p1], mine),
            "rc": (L[n0:n1], dd[s0:s1], q[s0:s1]),
            "timing": {k: v[p0:p1] for k, v in t.items()},
            "slack": {"slack": s["slack"][p0:p1], "ep_slack": s["ep_slack"][e0:e1],
                      "ep_order": s["ep_order"][:, e0:e1], "wns": wns[i], "tns": tns[i]},
            "ep_pin": gpu["ep_pin"][e0:e1] - p0,
        })
    return out


def _run_batch(designs, **opts):
    print(f"[batch] {len(designs)} designs, pins={sum(d.n_pins for d in designs)} opts={opts}", flush=True)
    b = STA(designs, **opts)
    b.update()
    g = run_gpu(b)
    offs = b.batch_offsets()
    wns, tns = b.batch_report()
    b.close()
    return split(designs, g, offs, wns, tns), offs


def _assert_same(a, b, where):
    for k in ("levels", "rc"):
        for x, y in zip(a[k], b[k]):
            assert np.array_equal(x, y), (where, k)
    for k, v in a["timing"].items():
        assert np.array_equal(v, b["timing"][k]), (where, k)
    for k in ("slack", "ep_slack", "ep_order", "wns", "tns"):
        assert np.array_equal(np.asarray(a["slack"][k]), np.asarray(b["slack"][k])), (where, k)
    assert np.array_equal(a["ep_pin"], b["ep_pin"]), (where, "ep_pin")


@pytest.mark.parametrize("sched", [STA_SCHED_PERSISTENT, STA_SCHED_PER_LEVEL, STA_SCHED_GRAPH, STA_SCHED_FLOW])
def test_batch_bit_identical_to_single_designs(sched):
    designs = _designs(6, 7_100_000, 200, 20_000)
    parts, offs = _run_batch(designs, sched=sched)
    assert offs[0][-1] == sum(d.n_pins for d in designs)
    for i, d in enumerate(designs):
        s = STA(d, sched=sched)
        s.update()
        g = run_gpu(s)
        s.close()
        g["slack"]["wns"] = np.asarray(g["slack"]["wns"])
        g["slack"]["tns"] = np.asarray(g["slack"]["tns"])
        _assert_same(parts[i], g, f"design {i}")


def test_batch_matches_oracle_per_design():
    designs = _designs(5, 7_200_000, 100, 8_000)
    parts, _ = _run_batch(designs)
    for i, d in enumerate(designs):
        r = oracle.sta(d)
        compare_full(d, r, parts[i])


def test_batch_with_wide_nets_and_one_design():
    """A batch of one design equals the design alone; a batch whose designs
    carry high-fanout nets routes them through the wide-net kernel."""
    cfgs = [synth.mid_config(seed=31 + i, n_cells=3000 + 1000 * i, n_levels=12 + i, n_hf=2, hf_min=300,
                             hf_max=600, lib_seed=77) for i in range(3)]
    designs = [synth.generate(c) for c in cfgs]
    parts, _ = _run_batch(designs)
    for i, d in enumerate(designs):
        compare_full(d, oracle.sta(d), parts[i])
    one, _ = _run_batch(designs[:1])
    s = STA(designs[0])
    s.update()
    g = run_gpu(s)
    s.close()
    _assert_same(one[0], g, "single")


def _single(d, **opts):
    s = STA(d, **opts)
    s.update()
    g = run_gpu(s)
    s.close()
    g["slack"]["wns"] = np.asarray(g["slack"]["wns"])
    g["slack"]["tns"] = np.asarray(g["slack"]["tns"])
    return g


@pytest.mark.parametrize("sched", [STA_SCHED_PERSISTENT, STA_SCHED_PER_LEVEL, STA_SCHED_GRAPH])
def test_corner_batch(sched):
    """One netlist under four libraries (corners) as one batch of per-design
    libraries: each corner bit for bit as the netlist timed alone with that
    library, and element by element against the FP64 oracle."""
    cfgs = synth.corner_configs(synth.mid_config(n_cells=20_000, n_levels=25, seed=41, n_hf=2, hf_min=300,
                                                 hf_max=900))
    designs = [synth.generate(c) for c in cfgs]
    assert np.array_equal(designs[0].net_sink_pin, designs[3].net_sink_pin)
    assert not np.array_equal(designs[0].tables, designs[3].tables)
    parts, _ = _run_batch(designs, sched=sched)
    for i, d in enumerate(designs):
        _assert_same(parts[i], _single(d, sched=sched), f"corner {i}")
        if sched == STA_SCHED_PER_LEVEL:
            compare_full(d, oracle.sta(d), parts[i])
    # the corners differ (different libraries give different arrivals)
    assert not np.array_equal(parts[0]["timing"]["at"], parts[3]["timing"]["at"])


def test_mixed_library_batch():
    """Uneven designs each with one of three libraries (shared by designs
    with the same one): per design bit for bit as alone and against the
    oracle."""
    cfgs = synth.mixed_batch_configs(9, n_libs=3, base_seed=7_400_000, min_cells=200, max_cells=12_000)
    designs = [synth.generate(c) for c in cfgs]
    parts, _ = _run_batch(designs)
    for i, d in enumerate(designs):
        _assert_same(parts[i], _single(d), f"design {i}")
        compare_full(d, oracle.sta(d), parts[i])


def test_batch_autotune_and_wire_caps():
    designs = _designs(4, 7_300_000, 500, 10_000)
    b = STA(designs)
    r = b.autotune(reps=2)
    assert r.n_tried >= 3 and r.sched in (STA_SCHED_PERSISTENT, STA_SCHED_PER_LEVEL, STA_SCHED_GRAPH, STA_SCHED_FLOW)
    assert r.ms > 0
    print(f"[batch] autotune sched={r.sched} blocks={r.sweep_blocks} ms={r.ms:.3f}", flush=True)
    # new caps through the union node order reach every design: each design's
    # figures equal those of the design alone with the same caps
    pin_off, ep_off, node_off = b.batch_offsets()
    assert node_off[-1] == sum(int(d.n_nodes) for d in designs)
    caps = [(d.cap_ff * 1.5).astype(np.float32) for d in designs]
    b.set_wire_caps(np.concatenate(caps))
    b.update()
    wns, tns = b.batch_report()
    b.close()
    for i, d in enumerate(designs):
        s = STA(d)
        s.set_wire_caps(caps[i])
        s.update()
        r = s.slack()
        s.close()
        assert np.array_equal(wns[i], r["wns"]) and np.array_equal(tns[i], r["tns"]), (i, wns[i], r["wns"])


# The benchmark's batch: 256 uneven designs (1k-200k cells, 10-80 levels,
# 29M pins in all), run once as a union in the graph schedule the benchmark's
# autotuner picks and once per level; every design's slice is then compared
# bit for bit with the design timed alone and element by element with the
# FP64 oracle, in groups of 32 designs per test.
_BENCH_BATCH = {}
_GROUPS = 8


def _bench_batch():
    if not _BENCH_BATCH:
        designs = [synth.generate(c) for c in synth.batch_configs(256)]
        parts, offs = _run_batch(designs, sched=STA_SCHED_GRAPH)
        parts_pl, _ = _run_batch(designs, sched=STA_SCHED_PER_LEVEL)
        for i in range(len(designs)):
            _assert_same(parts[i], parts_pl[i], f"design {i}: graph vs per-level batch")
        _BENCH_BATCH.update(designs=designs, parts=parts)
    return _BENCH_BATCH


@pytest.mark.slow
@pytest.mark.parametrize("group", range(_GROUPS))
def test_bench_batch_256(group):
    b = _bench_batch()
    designs, parts = b["designs"], b["parts"]
    per = len(designs) // _GROUPS
    for i in range(group * per, (group + 1) * per):
        d = designs[i]
        s = STA(d, sched=STA_SCHED_GRAPH)
        s.update()
        g = run_gpu(s)
        s.close()
        g["slack"]["wns"] = np.asarray(g["slack"]["wns"])
        g["slack"]["tns"] = np.asarray(g["slack"]["tns"])
        _assert_same(parts[i], g, f"design {i}")
        compare_full(d, oracle.sta(d), parts[i])
    print(f"[batch] designs {group * per}..{(group + 1) * per - 1} of the 256-design batch ok", flush=True)
