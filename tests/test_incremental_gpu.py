"""GPU incremental update: after the caps of a few nets change,
sta_update_timing_incremental must leave every reported value bitwise equal
to a full sta_update_timing with the same caps (chained incremental calls
against a second context doing full updates), and within the FP64 oracle's
tolerance.  Covers one net, a handful, a tenth of the nets, duplicates, an
empty list, PI-driven and high-fanout (split) drivers, wide RC nets, the
smooth mode, a device-resident list and the error paths."""
import numpy as np
import pytest

import oracle
from paper_2511_11660_amd import synth
from paper_2511_11660_amd.sta import STA, STA_E_ARG, STA_E_STATE, StaError
from parity import compare_full, run_gpu

pytestmark = pytest.mark.gpu


def _bits(a):
    a = np.ascontiguousarray(a)
    return a.view(np.uint32) if a.dtype == np.float32 else a


def _assert_same(got, ref, where):
    for grp in ("rc", "timing", "slack"):
        g, r = got[grp], ref[grp]
        items = g.items() if isinstance(g, dict) else enumerate(g)
        for k, v in items:
            if v is None:
                continue
            w = r[k]
            if isinstance(v, np.ndarray):
                if v.dtype == np.float64:
                    ok = np.array_equal(v.view(np.uint64), w.view(np.uint64))
                else:
                    ok = np.array_equal(_bits(v), _bits(w))
                if not ok:
                    diff = np.argwhere(_bits(v) != _bits(w)) if v.dtype != np.float64 else "fp64"
                    raise AssertionError(f"{where}: {grp}.{k} differs at {diff[:5] if not isinstance(diff, str) else diff}")
            else:
                assert v == w, (where, grp, k)


def _snapshot(s):
    out = run_gpu(s)
    out.pop("levels")
    out.pop("ep_pin")
    return out


def _perturb(d, caps, nets, rng):
    caps = caps.copy()
    for n in nets:
        a, b = int(d.net_node_ptr[n]), int(d.net_node_ptr[n + 1])
        caps[a:b] = (caps[a:b] * rng.uniform(0.3, 3.0, b - a)).astype(np.float32)
    return caps


def _chain(d, sizes, seed, check_oracle=True, **opts):
    """Incremental calls on one context against full updates on another."""
    rng = np.random.default_rng(seed)
    inc = STA(d, **opts)
    full = STA(d, **opts)
    inc.update()
    caps = d.cap_ff.astype(np.float32).copy()
    for i, k in enumerate(sizes):
        nets = rng.choice(d.n_nets, size=k, replace=False) if k else np.zeros(0, np.int32)
        print(f"[inc] pins={d.n_pins} step={i} nets={k}", flush=True)
        caps = _perturb(d, caps, nets, rng)
        inc.set_wire_caps(caps)
        inc.update_incremental(nets.astype(np.int32))
        full.set_wire_caps(caps)
        full.update()
        _assert_same(_snapshot(inc), _snapshot(full), f"step {i} ({k} nets)")
    if check_oracle:
        r = oracle.sta(d, wire_cap=caps.astype(np.float64))
        compare_full(d, r, run_gpu(inc))
    inc.close()
    full.close()


# blocks = 1: a one-block queued sweep, which hands over to per-phase launches
# at the first phase with more than 16 items; both schedules and the
# hand-over are covered
@pytest.mark.parametrize("blocks", [0, 1])
def test_incremental_tiny_chain(blocks):
    d = synth.generate(synth.tiny_config(seed=31, dangling_policy=1))
    _chain(d, [1, 1, 5, 40, 0, d.n_nets // 10, d.n_nets], seed=1, sweep_blocks=blocks)


def test_incremental_wide_rc_nets():
    """Every net above 40 RC nodes goes through the wide-net RC kernel."""
    d = synth.generate(synth.tiny_config(seed=32))
    _chain(d, [3, 30, 300], seed=2, big_net_nodes=40)


@pytest.mark.parametrize("blocks", [0, 1])
def test_incremental_mid_design(blocks):
    d = synth.generate(synth.mid_config(n_cells=60_000, n_levels=40, seed=33))
    _chain(d, [1, 10, 100, 3000], seed=3, sweep_blocks=blocks)


def test_incremental_benchmark_design():
    """The incremental measurement's own workload: the 10M-pin design after 1,
    100 and 10,000 nets are re-capped, each bitwise a full update with the same
    caps (10,000 nets goes past the full-update threshold), the last also
    against the oracle."""
    d = synth.generate(synth.large_config())
    _chain(d, [1, 100, 10_000], seed=4)


@pytest.mark.parametrize("blocks", [0, 1])
def test_incremental_split_high_fanout_drivers(blocks):
    cfg = synth.mid_config(seed=34, n_cells=8_000, n_levels=12, n_hf=3, hf_min=1500, hf_max=3000)
    d = synth.generate(cfg)
    hf = np.argsort(np.diff(d.net_sink_ptr))[-3:]  # the high-fanout nets themselves
    rng = np.random.default_rng(4)
    inc, full = STA(d, sweep_blocks=blocks), STA(d, sweep_blocks=blocks)
    inc.update()
    caps = d.cap_ff.astype(np.float32).copy()
    for i, nets in enumerate([hf[:1], hf, np.concatenate([hf, rng.choice(d.n_nets, 50, replace=False)])]):
        caps = _perturb(d, caps, nets, rng)
        inc.set_wire_caps(caps)
        inc.update_incremental(nets.astype(np.int32))
        full.set_wire_caps(caps)
        full.update()
        _assert_same(_snapshot(inc), _snapshot(full), f"step {i}")
    inc.close()
    full.close()


def test_incremental_duplicates_pi_nets_and_device_list():
    import torch
    d = synth.generate(synth.tiny_config(seed=35))
    drv_kind = np.asarray(d.pin_kind)[np.asarray(d.net_driver)]
    pi_nets = np.flatnonzero(drv_kind == 0)[:5]
    rng = np.random.default_rng(5)
    inc, full = STA(d), STA(d)
    inc.update()
    caps = _perturb(d, d.cap_ff.astype(np.float32), pi_nets, rng)
    inc.set_wire_caps(caps)
    lst = np.concatenate([pi_nets, pi_nets, pi_nets[:2]]).astype(np.int32)
    inc.update_incremental(torch.from_numpy(lst).cuda())
    full.set_wire_caps(caps)
    full.update()
    _assert_same(_snapshot(inc), _snapshot(full), "pi nets")
    before = _snapshot(inc)
    inc.update_incremental(np.zeros(0, np.int32))
    _assert_same(_snapshot(inc), before, "empty list")
    inc.close()
    full.close()


@pytest.mark.parametrize("blocks", [0, 1])
def test_incremental_smooth_mode(blocks):
    d = synth.generate(synth.mid_config(n_cells=20_000, n_levels=25, seed=36))
    rng = np.random.default_rng(6)
    inc = STA(d, mode=1, gamma_ps=5.0, sweep_blocks=blocks)
    full = STA(d, mode=1, gamma_ps=5.0, sweep_blocks=blocks)
    inc.update()
    caps = d.cap_ff.astype(np.float32).copy()
    for k in (1, 50, 2000):
        nets = rng.choice(d.n_nets, k, replace=False)
        caps = _perturb(d, caps, nets, rng)
        inc.set_wire_caps(caps)
        inc.update_incremental(nets.astype(np.int32))
        full.set_wire_caps(caps)
        full.update()
        a, b = inc.timing(), full.timing()
        for key in ("at", "slew", "crit"):
            np.testing.assert_array_equal(_bits(a[key]), _bits(b[key]))
        sa, sb = inc.slack(), full.slack()
        np.testing.assert_array_equal(_bits(sa["ep_slack"]), _bits(sb["ep_slack"]))
        assert sa["tns"].tobytes() == sb["tns"].tobytes() and sa["wns"].tobytes() == sb["wns"].tobytes()
    inc.close()
    full.close()


def test_incremental_errors():
    d = synth.generate(synth.tiny_config(seed=37))
    s = STA(d)
    with pytest.raises(StaError) as e:
        s.update_incremental(np.array([0], np.int32))
    assert e.value.status == STA_E_STATE
    s.update()
    with pytest.raises(StaError) as e:
        s.update_incremental(np.array([d.n_nets], np.int32))
    assert e.value.status == STA_E_ARG
    with pytest.raises(StaError) as e:
        s.update_incremental(np.array([-1], np.int32))
    assert e.value.status == STA_E_ARG
    s.close()
