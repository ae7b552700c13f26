"""GPU parity: the HIP path through the C ABI against the FP64 oracle, element
by element, on seeded synthetic designs (tiny, mid-size, 1M pins) and on the
10M-pin design the benchmark times, plus hand-built and edge-case designs."""
import numpy as np
import pytest

import oracle
from designs import CIN, COUT, PI, PO, make_design, planar_table, single_segment_net
from paper_2511_11660_amd import synth
from paper_2511_11660_amd.sta import STA, STA_SCHED_FLOW, STA_SCHED_GRAPH, STA_SCHED_PER_LEVEL, STA_SCHED_PERSISTENT
from parity import assert_bitwise_equal, compare_full, magnitude_scales, run_gpu

pytestmark = pytest.mark.gpu


def _run(d, **opts):
    print(f"[parity] design pins={d.n_pins} cells={d.n_cells} opts={opts}", flush=True)
    s = STA(d, **opts)
    s.update()
    out = run_gpu(s)
    s.close()
    return out


@pytest.mark.parametrize("sched", [STA_SCHED_PERSISTENT, STA_SCHED_PER_LEVEL, STA_SCHED_GRAPH, STA_SCHED_FLOW])
def test_tiny(sched):
    d = synth.generate(synth.tiny_config())
    r = oracle.sta(d)
    stats = compare_full(d, r, _run(d, sched=sched))
    print(stats)


def test_tiny_shuffled_ids_and_big_net_path():
    """Permuted pin, cell and net ids; every net with more than 8 RC nodes goes
    through the wide-net RC kernel (preorder layout)."""
    d = synth.generate(synth.tiny_config(seed=7, shuffle=1))
    r = oracle.sta(d)
    compare_full(d, r, _run(d, big_net_nodes=8))


def test_tiny_dangling_endpoints():
    d = synth.generate(synth.tiny_config(seed=9, dangling_policy=1, rat_early_ps=40.0))
    r = oracle.sta(d)
    compare_full(d, r, _run(d))


def test_worked_chain_design():
    import test_oracle_pins as pins
    d, *_ = pins._chain_design()
    r = oracle.sta(d)
    compare_full(d, r, _run(d))


def test_high_fanout_nets():
    """Nets of a few hundred to a thousand sinks driven by PIs / level-1 cells
    (the RC trees exceed the LDS-staged limit)."""
    cfg = synth.mid_config(seed=21, n_cells=20_000, n_levels=25, n_hf=6, hf_min=200, hf_max=1000)
    d = synth.generate(cfg)
    assert np.diff(d.net_node_ptr).max() > 255
    r = oracle.sta(d)
    compare_full(d, r, _run(d))


@pytest.mark.parametrize("sched", [STA_SCHED_PERSISTENT, STA_SCHED_PER_LEVEL, STA_SCHED_GRAPH, STA_SCHED_FLOW])
def test_mid(sched):
    d = synth.generate(synth.mid_config(n_cells=60_000, n_levels=40, seed=12))
    r = oracle.sta(d)
    compare_full(d, r, _run(d, sched=sched))


def test_mid_every_schedule_bitwise():
    """A 40-level design with high-fanout nets: every (schedule, overlap)
    pair against the oracle and bit for bit against each other."""
    _all_schedules(synth.generate(synth.mid_config(n_cells=30_000, n_levels=40, seed=25, n_hf=4, hf_min=1100,
                                                   hf_max=2500)))


# (schedule, overlap): the persistent sweeps; per-level launches and their
# graph, each with every phase in stream order and with the RC groups and the
# reduction on side streams; the dataflow sweeps
SCHEDS = ((STA_SCHED_PERSISTENT, 0), (STA_SCHED_PER_LEVEL, 0), (STA_SCHED_PER_LEVEL, 1), (STA_SCHED_GRAPH, 0),
          (STA_SCHED_GRAPH, 1), (STA_SCHED_FLOW, 0))


def _all_schedules(d):
    """Every schedule on one design: each against the FP64 oracle element by
    element, and all of them bit-identical to each other (same per-pin
    arithmetic in every schedule)."""
    r = oracle.sta(d)
    scales = magnitude_scales(d, r)
    first = None
    for sched, ov in SCHEDS:
        g = _run(d, sched=sched, overlap=ov)
        print(f"[parity] sched={sched} overlap={ov}", compare_full(d, r, g, scales=scales), flush=True)
        if first is None:
            first = g
        else:
            assert_bitwise_equal(first, g, f"schedule {sched}/{ov} vs {SCHEDS[0]}")


@pytest.mark.slow
def test_1m_pins_every_schedule():
    _all_schedules(synth.generate(synth.mid_config()))


def test_determinism_and_repeat():
    d = synth.generate(synth.mid_config(n_cells=30_000, n_levels=30, seed=13))
    s = STA(d)
    s.update()
    a = run_gpu(s)
    s.update()
    s.update()
    b = run_gpu(s)
    s.close()
    for k in ("at", "slew", "rat", "crit"):
        np.testing.assert_array_equal(a["timing"][k], b["timing"][k])
    np.testing.assert_array_equal(a["slack"]["slack"], b["slack"]["slack"])
    np.testing.assert_array_equal(a["slack"]["tns"], b["slack"]["tns"])
    np.testing.assert_array_equal(a["slack"]["ep_order"], b["slack"]["ep_order"])


def test_set_wire_caps_host_and_device():
    import torch
    d = synth.generate(synth.tiny_config(seed=3))
    rng = np.random.default_rng(0)
    caps = (d.cap_ff * rng.uniform(0.5, 2.0, d.cap_ff.shape)).astype(np.float32)
    r = oracle.sta(d, wire_cap=caps.astype(np.float64))
    s = STA(d)
    s.set_wire_caps(caps)
    s.update()
    compare_full(d, r, run_gpu(s))
    caps2 = (d.cap_ff * rng.uniform(0.5, 2.0, d.cap_ff.shape)).astype(np.float32)
    r2 = oracle.sta(d, wire_cap=caps2.astype(np.float64))
    s.set_wire_caps(torch.from_numpy(caps2).cuda())
    torch.cuda.synchronize()
    s.update()
    compare_full(d, r2, run_gpu(s))
    s.close()


def test_device_outputs_match_host_outputs():
    import torch
    from paper_2511_11660_amd import sta as S
    d = synth.generate(synth.tiny_config(seed=4))
    s = STA(d)
    s.update()
    h = s.timing()
    at = torch.empty((d.n_pins, 4), dtype=torch.float32, device="cuda")
    crit = torch.empty((d.n_pins, 4), dtype=torch.int8, device="cuda")
    S.sta_report_timing(s.ctx, at=at, crit=crit, dst=S.STA_DEVICE)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(at.cpu().numpy(), h["at"])
    np.testing.assert_array_equal(crit.cpu().numpy(), h["crit"])
    s.close()


def test_single_cell_and_pi_to_po():
    """Degenerate designs: one cell; a PI wired straight to a PO; a dangling PI."""
    kinds = [PI, PI, PI, CIN, COUT, PO, PO]
    cells = [(0, [3], 4)]
    nets = [single_segment_net(0, [3], 0.01, 1.0), single_segment_net(1, [6], 0.02, 0.5),
            single_segment_net(2, [], 0.0, 0.0), single_segment_net(4, [5], 0.03, 2.0)]
    tables = np.stack([np.stack([planar_table(7, 0.1, 1.3)] * 2 + [planar_table(3, 0.05, 2.0)] * 2)])
    d = make_design(kinds, cells, nets, n_inputs=[1], sense=[2], pin_cap=[1.0], tables=tables)
    r = oracle.sta(d)
    compare_full(d, r, _run(d))


@pytest.mark.slow
def test_10m_pins_every_schedule():
    """The benchmark's 10M-pin design at full size in every schedule, the
    benchmark's own (per level, or its graph) included."""
    _all_schedules(synth.generate(synth.large_config()))


def _wide_cell_design(seed=11):
    """Cells of 5 and 6 inputs (beyond the inline fanin record, so the sweeps
    read fanins through the CSR), mixed with 1- and 2-input cells, over three
    levels, every output net a multi-sink star."""
    rng = np.random.default_rng(seed)
    n_inputs = [1, 2, 5, 6]
    kinds, cells, nets = [], [], []

    def pin(kind):
        kinds.append(kind)
        return len(kinds) - 1

    pis = [pin(PI) for _ in range(10)]
    sinks_of = {p: [] for p in pis}
    prev = list(pis)
    for level in range(3):
        outs = []
        for _ in range(6):
            t = int(rng.integers(0, 4))
            srcs = rng.choice(prev + pis, size=n_inputs[t], replace=True)
            ins = []
            for src in srcs:
                ci = pin(CIN)
                sinks_of[int(src)].append(ci)
                ins.append(ci)
            o = pin(COUT)
            sinks_of[o] = []
            cells.append((t, ins, o))
            outs.append(o)
        prev = outs
    for o in prev:
        sinks_of[o].append(pin(PO))
    for drv, sk in sinks_of.items():
        nets.append(single_segment_net(drv, sk, float(rng.uniform(0.005, 0.05)), float(rng.uniform(0.2, 2.0))))
    tables = np.stack([np.stack([planar_table(5 + 3 * t, 0.1, 1.0 + 0.2 * t, 0.001),
                                 planar_table(6 + 2 * t, 0.12, 1.1, 0.002),
                                 planar_table(3, 0.05 + 0.01 * t, 2.0),
                                 planar_table(4, 0.06, 1.8 + 0.1 * t)]) for t in range(4)])
    return make_design(kinds, cells, nets, n_inputs=n_inputs, sense=[1, 0, 2, 1], pin_cap=[1.0, 1.5, 0.8, 2.2],
                       tables=tables, po_rat=40.0, rat_early=20.0)


@pytest.mark.parametrize("sched", [STA_SCHED_PERSISTENT, STA_SCHED_PER_LEVEL])
def test_cells_wider_than_inline_fanins(sched):
    d = _wide_cell_design()
    assert int(np.diff(d.cell_in_ptr).max()) > 4
    r = oracle.sta(d)
    compare_full(d, r, _run(d, sched=sched))


@pytest.mark.parametrize("sched", [STA_SCHED_PERSISTENT, STA_SCHED_PER_LEVEL, STA_SCHED_GRAPH])
def test_split_high_fanout_drivers(sched):
    """Drivers of 1.5k-5k sinks: each gets a chunk of its own and its sinks
    beyond the first piece go to separate work items (forward sink states,
    backward RAT merges folded into the driver)."""
    cfg = synth.mid_config(seed=23, n_cells=20_000, n_levels=20, n_hf=4, hf_min=1500, hf_max=5000)
    d = synth.generate(cfg)
    assert np.diff(d.net_sink_ptr).max() > 1024
    r = oracle.sta(d)
    compare_full(d, r, _run(d, sched=sched))
