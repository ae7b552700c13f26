"""GPU RC estimation from pin positions (sta_estimate_rc) against the oracle
(oracle/rc_estimate.py): every output bitwise equal, since both sides take
the same FP32 distance decisions and the same FP32 products.  Covers a
generated design, a fanout ladder across the lane-per-net / wave-per-net /
block-per-net splits (8 and 64 pins) up to the largest supported net, integer-grid and
coincident positions (distance ties everywhere), device-resident inputs,
sampled checks on 1.2M- and 12M-pin designs, timing on the estimated trees,
and the error paths.  Then the gradient to positions through the trees
(sta_estimate_rc_backward) against the oracle's, alone on random node
gradients and chained after the smooth timing adjoint."""
from types import SimpleNamespace

import numpy as np
import pytest

import oracle
from oracle import rc_estimate as R
from paper_2511_11660_amd import synth
from paper_2511_11660_amd.sta import (STA, STA_E_ARG, STA_E_UNSUPPORTED, STA_DEVICE, StaError, estimate_rc,
                                      estimate_rc_backward, sta_estimate_rc, sta_graph_desc, sta_wire_params)
from parity import compare_full, run_gpu

pytestmark = pytest.mark.gpu

WIRE = (0.0021, 0.0017, 0.19, 0.23)  # r_x, r_y (kOhm/um), c_x, c_y (fF/um)
KEYS = ("net_node_ptr", "parent", "res_kohm", "cap_ff", "sink_node")


def _bits(a):
    a = np.ascontiguousarray(a)
    return a.view(np.uint32) if a.dtype == np.float32 else a


def _assert_same(got, ref):
    for k in KEYS:
        g = got[k].cpu().numpy() if hasattr(got[k], "cpu") else got[k]
        assert g.shape == ref[k].shape, k
        bad = np.flatnonzero(_bits(g) != _bits(ref[k]))
        assert bad.size == 0, f"{k} differs at {bad[:8].tolist()}: {g[bad[:4]]} vs {ref[k][bad[:4]]}"


def _nets(fanouts, seed=0):
    """Netlist-only object: net i has its own driver pin and fanouts[i] sink
    pins, the sinks of all nets shuffled over the pin ids."""
    rng = np.random.default_rng(seed)
    fo = np.asarray(fanouts, np.int64)
    n_pins = int(len(fo) + fo.sum())
    perm = rng.permutation(n_pins).astype(np.int32)
    ptr = np.zeros(len(fo) + 1, np.int32)
    ptr[1:] = np.cumsum(fo)
    return SimpleNamespace(n_pins=n_pins, n_cells=0, n_nets=len(fo), n_pi=0, n_po=0, n_sinks=int(ptr[-1]),
                           net_driver=perm[: len(fo)], net_sink_ptr=ptr, net_sink_pin=perm[len(fo):])


def test_tiny_design_bitwise():
    d = synth.generate(synth.tiny_config(seed=5))
    x, y = synth.place(d, seed=2)
    _assert_same(estimate_rc(d, x, y, *WIRE), R.estimate_rc(d, x, y, *WIRE))


LADDER = [0, 1, 2, 3, 6, 7, 8, 9, 31, 62, 63, 64, 65, 100, 511, 1023, 1024, 1025, 2047, 3000, 6000, 12287]


@pytest.mark.parametrize("kind", ["uniform", "grid", "coincident"])
def test_fanout_ladder_bitwise(kind):
    d = _nets(LADDER + [5] * 50, seed=len(kind))
    rng = np.random.default_rng(11)
    if kind == "uniform":
        x = rng.uniform(0.0, 500.0, d.n_pins).astype(np.float32)
        y = rng.uniform(0.0, 500.0, d.n_pins).astype(np.float32)
    elif kind == "grid":  # distances tie all the time
        x = rng.integers(0, 9, d.n_pins).astype(np.float32) * 2.5
        y = rng.integers(0, 9, d.n_pins).astype(np.float32) * 2.5
    else:  # two clusters of identical positions: zero-length wires and ties at 0
        c = rng.integers(0, 2, d.n_pins)
        x = np.where(c == 0, 10.0, 70.0).astype(np.float32)
        y = np.where(c == 0, 5.0, 5.0).astype(np.float32)
    _assert_same(estimate_rc(d, x, y, *WIRE), R.estimate_rc(d, x, y, *WIRE))


def test_device_inputs_match_host():
    import torch
    d = _nets([0, 4, 70, 1500, 9, 63, 64], seed=3)
    rng = np.random.default_rng(4)
    x = rng.uniform(-50.0, 50.0, d.n_pins).astype(np.float32)
    y = rng.uniform(-50.0, 50.0, d.n_pins).astype(np.float32)
    ref = R.estimate_rc(d, x, y, *WIRE)
    # positions on the device, net CSR on the host
    _assert_same(estimate_rc(d, torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda(), *WIRE), ref)
    # everything on the device, through the C entry point
    dev = {k: torch.from_numpy(np.ascontiguousarray(getattr(d, k))).cuda()
           for k in ("net_driver", "net_sink_ptr", "net_sink_pin")}
    g = sta_graph_desc(d.n_pins, 0, d.n_nets, 0, 0, None, None, None, None, None, dev["net_driver"].data_ptr(),
                       dev["net_sink_ptr"].data_ptr(), dev["net_sink_pin"].data_ptr(), STA_DEVICE)
    nn = d.n_nets + 3 * d.n_sinks
    out = {"net_node_ptr": torch.zeros(d.n_nets + 1, dtype=torch.int64, device="cuda"),
           "parent": torch.zeros(nn, dtype=torch.int32, device="cuda"),
           "res_kohm": torch.zeros(nn, dtype=torch.float32, device="cuda"),
           "cap_ff": torch.zeros(nn, dtype=torch.float32, device="cuda"),
           "sink_node": torch.zeros(d.n_sinks, dtype=torch.int32, device="cuda")}
    sta_estimate_rc(g, torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda(), sta_wire_params(*WIRE),
                    out["net_node_ptr"], out["parent"], out["res_kohm"], out["cap_ff"], out["sink_node"],
                    STA_DEVICE, torch.cuda.current_stream())
    _assert_same(out, ref)


@pytest.mark.parametrize("size", ["1M", "10M"])
def test_design_sampled(size):
    """1.2M and 12M pins (the second with positions in device memory, as the
    benchmark runs it): every net's node range by its closed form, the tree
    shape on all nets, and 3000 sampled nets bitwise against the oracle."""
    import torch
    d = synth.generate(synth.mid_config() if size == "1M" else synth.large_config())
    x, y = synth.place(d, seed=7)
    if size == "1M":
        got = estimate_rc(d, x, y, *WIRE)
    else:
        got = {k: v.cpu().numpy() for k, v in
               estimate_rc(d, torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda(), *WIRE).items()}
    nsp = np.asarray(d.net_sink_ptr, np.int64)
    np.testing.assert_array_equal(got["net_node_ptr"], np.arange(d.n_nets + 1) + 3 * nsp)
    ptr = got["net_node_ptr"]
    local = np.arange(ptr[-1]) - np.repeat(ptr[:-1], np.diff(ptr))
    par = got["parent"]
    assert np.all((par < local) & ((par >= 0) | (local == 0)) & ((local > 0) | (par == -1)))
    rng = np.random.default_rng(8)
    for n in rng.choice(d.n_nets, 3000, replace=False):
        pins = np.concatenate([[d.net_driver[n]], d.net_sink_pin[nsp[n]:nsp[n + 1]]])
        p, r, c, node_of = R.estimate_net(x[pins], y[pins], *WIRE)
        a, b = ptr[n], ptr[n + 1]
        assert np.array_equal(par[a:b], p) and np.array_equal(_bits(got["res_kohm"][a:b]), _bits(r)) \
            and np.array_equal(_bits(got["cap_ff"][a:b]), _bits(c)), f"net {n}"
        assert np.array_equal(got["sink_node"][nsp[n]:nsp[n + 1]], node_of[1:]), f"net {n}"


def test_timing_on_estimated_trees():
    """The estimated trees are a valid RC input: full timing on them matches
    the oracle's timing on the oracle's trees."""
    d = synth.generate(synth.tiny_config(seed=9))
    x, y = synth.place(d, seed=3)
    e = synth.with_rc(d, estimate_rc(d, x, y, *WIRE))
    t = STA(e, sched=1)
    t.update()
    compare_full(e, oracle.sta(synth.with_rc(d, R.estimate_rc(d, x, y, *WIRE))), run_gpu(t))
    t.close()


def test_no_nets_and_sinkless_nets():
    d = _nets([], seed=0)
    d.n_pins = 3
    got = estimate_rc(d, np.zeros(3, np.float32), np.zeros(3, np.float32), *WIRE)
    np.testing.assert_array_equal(got["net_node_ptr"], [0])
    d = _nets([0, 0, 0], seed=1)
    got = estimate_rc(d, np.arange(3, dtype=np.float32), np.zeros(3, np.float32), *WIRE)
    np.testing.assert_array_equal(got["net_node_ptr"], [0, 1, 2, 3])
    np.testing.assert_array_equal(got["parent"], [-1, -1, -1])


def _status(d, x, y):
    with pytest.raises(StaError) as e:
        estimate_rc(d, x, y, *WIRE)
    return e.value.status


def test_errors():
    d = _nets([3, 2], seed=2)
    x = np.zeros(d.n_pins, np.float32)
    y = np.zeros(d.n_pins, np.float32)
    bad = _nets([3, 2], seed=2)
    bad.net_sink_pin = bad.net_sink_pin.copy()
    bad.net_sink_pin[4] = d.n_pins
    assert _status(bad, x, y) == STA_E_ARG
    bad = _nets([3, 2], seed=2)
    bad.net_driver = bad.net_driver.copy()
    bad.net_driver[1] = -1
    assert _status(bad, x, y) == STA_E_ARG
    bad = _nets([3, 2], seed=2)
    bad.net_sink_ptr = np.array([0, 6, 5], np.int32)
    assert _status(bad, x, y) == STA_E_ARG
    xn = x.copy()
    xn[2] = np.nan
    assert _status(d, xn, y) == STA_E_ARG
    yi = y.copy()
    yi[0] = np.inf
    assert _status(d, x, yi) == STA_E_ARG
    yi[0] = -2e18  # finite, but distances could overflow
    assert _status(d, x, yi) == STA_E_ARG
    with pytest.raises(StaError) as e:
        estimate_rc(d, x, y, -1.0, 0.0, 0.0, 0.0)
    assert e.value.status == STA_E_ARG
    huge = _nets([12288], seed=0)
    z = np.zeros(huge.n_pins, np.float32)
    assert _status(huge, z, z) == STA_E_UNSUPPORTED
    # the library stays usable after the errors
    _assert_same(estimate_rc(d, x, y, *WIRE), R.estimate_rc(d, x, y, *WIRE))


# ------------------------------------------------------------ gradient to positions

def _grad_close(got, ref, what):
    g = got.cpu().numpy() if hasattr(got, "cpu") else got
    scale = 1e-5 * max(1.0, float(np.abs(ref).max()))
    err = np.abs(g.astype(np.float64) - ref)
    bad = np.flatnonzero(err > scale + 1e-5 * np.abs(ref))
    assert bad.size == 0, f"{what}: {bad[:5].tolist()} {g[bad[:3]]} vs {ref[bad[:3]]}"


@pytest.mark.parametrize("kind", ["design", "ladder", "grid"])
def test_position_gradient_matches_oracle(kind):
    """Random dJ/dR, dJ/dC per node through the trees: every tier (8-lane
    group, wave, block up to 12,287 sinks) against the FP64 oracle, and a
    second call bitwise equal to the first."""
    if kind == "design":
        d = synth.generate(synth.tiny_config(seed=4))
        x, y = synth.place(d, seed=5)
    else:
        d = _nets(LADDER + [5] * 30, seed=3)
        rng = np.random.default_rng(12)
        if kind == "ladder":
            x = rng.uniform(0.0, 300.0, d.n_pins).astype(np.float32)
            y = rng.uniform(0.0, 300.0, d.n_pins).astype(np.float32)
        else:  # coincident coordinates: zero-length segments, sgn(0) = 0
            x = rng.integers(0, 6, d.n_pins).astype(np.float32)
            y = rng.integers(0, 6, d.n_pins).astype(np.float32)
    rc = estimate_rc(d, x, y, *WIRE)
    nn = rc["parent"].size
    rng = np.random.default_rng(13)
    gR = rng.uniform(-1.0, 1.0, nn).astype(np.float32)
    gC = rng.uniform(-1.0, 1.0, nn).astype(np.float32)
    ox, oy = R.estimate_rc_backward(d, x, y, rc, *WIRE, gR, gC)
    gx, gy = estimate_rc_backward(d, x, y, rc, *WIRE, gR, gC)
    _grad_close(gx, ox, "dJ/dx")
    _grad_close(gy, oy, "dJ/dy")
    gx2, gy2 = estimate_rc_backward(d, x, y, rc, *WIRE, gR, gC)
    assert np.array_equal(gx.view(np.uint32), gx2.view(np.uint32))
    assert np.array_equal(gy.view(np.uint32), gy2.view(np.uint32))


def test_position_gradient_device_arrays():
    import torch
    d = _nets([0, 3, 12, 70, 2000], seed=9)
    rng = np.random.default_rng(14)
    x = rng.uniform(0.0, 80.0, d.n_pins).astype(np.float32)
    y = rng.uniform(0.0, 80.0, d.n_pins).astype(np.float32)
    rc = estimate_rc(d, x, y, *WIRE)
    gR = rng.uniform(-1.0, 1.0, rc["parent"].size).astype(np.float32)
    gC = rng.uniform(-1.0, 1.0, rc["parent"].size).astype(np.float32)
    hx, hy = estimate_rc_backward(d, x, y, rc, *WIRE, gR, gC)
    cu = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    dx, dy = estimate_rc_backward(d, cu(x), cu(y), {k: cu(v) for k, v in rc.items()}, *WIRE, cu(gR), cu(gC))
    assert np.array_equal(dx.cpu().numpy().view(np.uint32), hx.view(np.uint32))
    assert np.array_equal(dy.cpu().numpy().view(np.uint32), hy.view(np.uint32))


def test_timing_gradient_reaches_positions():
    """Positions -> estimated trees -> smooth timing -> adjoint -> position
    gradient, against the same chain through the FP64 oracle."""
    gamma = 5.0
    d = synth.generate(synth.tiny_config(seed=10, dangling_policy=1))
    x, y = synth.place(d, seed=4)
    rc = estimate_rc(d, x, y, *WIRE)
    e = synth.with_rc(d, rc)
    t = STA(e, mode=1, gamma_ps=gamma, sched=1)
    t.update()
    g = t.backward(1.0, 0.0)
    t.close()
    gx, gy = estimate_rc_backward(d, x, y, rc, *WIRE, g["grad_wire_res"], g["grad_wire_cap"])
    o = oracle.smooth_adjoint(synth.with_rc(d, R.estimate_rc(d, x, y, *WIRE)), gamma, 1.0, 0.0)
    ox, oy = R.estimate_rc_backward(d, x, y, rc, *WIRE, o["grad_wire_res"], o["grad_wire_cap"])
    for got, ref in ((gx, ox), (gy, oy)):
        scale = 1e-4 * max(1.0, float(np.abs(ref).max()))
        assert np.all(np.abs(got - ref) <= scale + 1e-3 * np.abs(ref))
    assert np.abs(ox).max() > 0


def test_position_gradient_rejects_a_foreign_tree():
    d = _nets([3, 2, 70], seed=5)
    rng = np.random.default_rng(1)
    x = rng.uniform(0.0, 10.0, d.n_pins).astype(np.float32)
    y = rng.uniform(0.0, 10.0, d.n_pins).astype(np.float32)
    rc = estimate_rc(d, x, y, *WIRE)
    z = np.zeros(rc["parent"].size, np.float32)
    for key, idx in (("sink_node", 0), ("sink_node", 4), ("parent", 1), ("parent", 13), ("parent", 200)):
        bad = {k: v.copy() for k, v in rc.items()}
        bad[key][idx] = bad[key][idx] + 1 if bad[key][idx] < 2 else bad[key][idx] - 1  # still in range, not the tree
        with pytest.raises(StaError) as e:
            estimate_rc_backward(d, x, y, bad, *WIRE, z, z)
        assert e.value.status == STA_E_ARG, (key, idx)
