"""GPU reduced-order (Arnoldi) net delays (sta_options.delay_model = 1)
against the FP64 oracle (oracle/arnoldi.py): full timing parity on the tiny
designs with the reduced-order delays fed to the oracle's propagation, through
the small-net and the wide-net RC kernels and every schedule; sampled sink
delays on a 1.2M-pin design; an incremental update bitwise equal to a full
one; and single-segment nets, where the reduced model is exact (R C ln 2)."""
import numpy as np
import pytest

import oracle
from oracle import arnoldi as AR
from paper_2511_11660_amd import synth
from paper_2511_11660_amd.sta import STA, STA_SCHED_GRAPH, STA_SCHED_PER_LEVEL, STA_SCHED_PERSISTENT
from parity import check_close, compare_full, run_gpu

pytestmark = pytest.mark.gpu


def _run(d, **opts):
    print(f"[arnoldi] pins={d.n_pins} opts={opts}", flush=True)
    s = STA(d, delay_model=1, **opts)
    s.update()
    out = run_gpu(s)
    s.close()
    return out


@pytest.mark.parametrize("sched", [STA_SCHED_PERSISTENT, STA_SCHED_PER_LEVEL, STA_SCHED_GRAPH])
def test_tiny_reduced_order_timing(sched):
    d = synth.generate(synth.tiny_config(seed=3))
    r = oracle.sta(d, sink_delay=AR.sink_delays(d))
    compare_full(d, r, _run(d, sched=sched))


def test_tiny_wide_net_path():
    """Every net above 16 RC nodes through the wide-net kernels (FP64 moments
    from the preorder scans, then the per-net reduction kernel)."""
    d = synth.generate(synth.tiny_config(seed=11, dangling_policy=1))
    r = oracle.sta(d, sink_delay=AR.sink_delays(d))
    compare_full(d, r, _run(d, sched=STA_SCHED_PER_LEVEL, big_net_nodes=16))


def test_single_segment_nets_are_rc_ln2():
    """The worked chain design's nets are single RC segments: the reduced
    model is one pole, so every sink delay is exactly R C^ ln 2 (the Elmore
    delay times ln 2), and the whole timing matches the oracle."""
    import test_oracle_pins as pins
    d, *_ = pins._chain_design()
    s = STA(d, delay_model=1, sched=STA_SCHED_PER_LEVEL)
    s.update()
    got = run_gpu(s)
    s.close()
    e = STA(d, sched=STA_SCHED_PER_LEVEL)
    e.update()
    _, de, _ = e.rc()
    e.close()
    np.testing.assert_allclose(got["rc"][1], de * np.log(2.0), rtol=1e-6)
    compare_full(d, oracle.sta(d, sink_delay=AR.sink_delays(d)), got)


@pytest.mark.parametrize("cfg", ["mid", "large"])
def test_sampled_delays(cfg):
    """1.2M and 12M pins (the benchmark's design): 2000 sampled nets' sink
    delays against the oracle's model, and on the large design also two nets
    above 255 nodes, which the wide-net kernels handle."""
    d = synth.generate(synth.mid_config() if cfg == "mid" else synth.large_config())
    print(f"[arnoldi] {cfg}: {d.n_pins} pins", flush=True)
    s = STA(d, delay_model=1, sched=STA_SCHED_PER_LEVEL)
    s.update()
    _, dr, _ = s.rc()
    s.close()
    nsp = np.asarray(d.net_sink_ptr)
    ptr = np.asarray(d.net_node_ptr)
    kind = np.asarray(d.pin_kind)
    cell_of = np.full(d.n_pins, -1)
    cell_of[np.asarray(d.cell_in_pin)] = np.repeat(np.arange(d.n_cells), np.diff(d.cell_in_ptr))
    rng = np.random.default_rng(2)
    nets = rng.choice(np.flatnonzero(np.diff(nsp) > 0), 2000, replace=False)
    if cfg == "large":  # and the two smallest wide nets (5k nodes: the dense oracle takes seconds each)
        m = np.diff(ptr)
        wide = np.flatnonzero((m > 255) & (np.diff(nsp) > 0))
        assert wide.size >= 2
        nets = np.concatenate([nets, wide[np.argsort(m[wide], kind="stable")[:2]]])
    got, ref = [], []
    for n in nets:
        a, b = ptr[n], ptr[n + 1]
        Chat = d.cap_ff[a:b].astype(np.float64)
        for sk in range(nsp[n], nsp[n + 1]):
            pin = d.net_sink_pin[sk]
            Chat[d.sink_node[sk]] += d.po_cap_ff if kind[pin] == 3 else d.pin_cap_ff[d.cell_type[cell_of[pin]]]
        ref.append(AR.net_delays(d.parent[a:b], d.res_kohm[a:b].astype(np.float64), Chat,
                                 d.sink_node[nsp[n]:nsp[n + 1]]))
        got.append(dr[nsp[n]:nsp[n + 1]])
    check_close("reduced-order sink delay", np.concatenate(got), np.concatenate(ref))


def test_incremental_update_with_reduced_order_delays():
    """Caps of a few nets change: the incremental update is bitwise the full
    update with the same caps, and both match the oracle."""
    d = synth.generate(synth.tiny_config(seed=17, dangling_policy=1))
    inc = STA(d, delay_model=1, sched=STA_SCHED_PER_LEVEL, big_net_nodes=16)
    full = STA(d, delay_model=1, sched=STA_SCHED_PER_LEVEL, big_net_nodes=16)
    inc.update()
    rng = np.random.default_rng(4)
    caps = d.cap_ff.astype(np.float32).copy()
    nets = rng.choice(d.n_nets, 12, replace=False).astype(np.int32)
    ptr = np.asarray(d.net_node_ptr)
    for n in nets:
        caps[ptr[n]:ptr[n + 1]] *= np.float32(1.7)
    inc.set_wire_caps(caps)
    full.set_wire_caps(caps)
    inc.update_incremental(nets)
    full.update()
    a, b = run_gpu(inc), run_gpu(full)
    inc.close()
    full.close()
    for grp in ("timing", "slack"):
        for k, v in a[grp].items():
            if isinstance(v, np.ndarray) and v.dtype != np.float64:
                assert np.array_equal(v.view(np.uint8), b[grp][k].view(np.uint8)), (grp, k)
    e = d.copy()
    e.cap_ff = caps
    compare_full(e, oracle.sta(e, sink_delay=AR.sink_delays(e)), a)
