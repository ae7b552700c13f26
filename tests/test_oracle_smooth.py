"""Pins for the smooth (differentiable) form of the FP64 oracle.

LSE bounds and the equal-input case, gamma -> 0 limits to the hard analysis,
every gradient of the FP64 adjoint (node caps, segment resistances, NLDM pin
loads, per-arc delays) against central finite differences of the FP64
objective (skipping steps that change a discrete choice), including the
differentiable configuration's 200 segments of the 1M-pin design, and the
integer special case of the arc-delay gradient."""
import numpy as np
import pytest

import oracle
from paper_2511_11660_amd import synth


@pytest.fixture(scope="module")
def small():
    return synth.generate(synth.mid_config(n_cells=3000, n_levels=15, seed=41))


def test_lse_bounds_and_equal_inputs(small):
    """max <= LSE_g <= max + g ln n per merge; with one-input cells and a
    positive-unate library every merge has a single candidate, so smooth late
    arrivals equal the hard ones exactly."""
    d = small
    hard = oracle.sta(d)
    for g in (5.0, 1.0):
        sm = oracle.smooth_sta(d, g)
        late_h, late_s = hard["at"][:, 2:], sm["at"][:, 2:]
        assert np.all(late_s >= late_h - 1e-9)
        # arrival gains at most g ln(#candidates) per level along a path
        assert np.all(late_s <= late_h + g * np.log(6) * hard["level"].max()[None] + 1e-9)
        np.testing.assert_array_equal(sm["at"][:, :2], hard["at"][:, :2])  # early stays hard


def test_gamma_to_zero_recovers_hard_tns_wns(small):
    d = small
    hard = oracle.sta(d)
    prev = None
    for g in (5.0, 0.5, 0.05, 0.005):
        sm = oracle.smooth_sta(d, g)
        err = abs(sm["tns"] - hard["tns"][1])
        if prev is not None:
            assert err <= prev + 1e-6
        prev = err
    assert prev < 1e-3 * max(1.0, abs(hard["tns"][1]))
    assert abs(oracle.smooth_sta(d, 0.005)["wns"] - hard["wns"][1]) < 0.05


def _fd_segments(d, n, seed):
    rng = np.random.default_rng(seed)
    nonroot = np.setdiff1d(np.arange(d.n_nodes), d.net_node_ptr[:-1])
    return rng.choice(nonroot, size=n, replace=False)


@pytest.mark.parametrize("g_tns,g_wns", [(1.0, 0.0), (0.0, 1.0), (0.7, 0.3)])
def test_adjoint_matches_central_differences(small, g_tns, g_wns):
    d, gamma, h = small, 5.0, 1e-3
    base = d.cap_ff.astype(np.float64)
    adj = oracle.smooth_adjoint(d, gamma, g_tns, g_wns, wire_cap=base)
    J = lambda r: g_tns * r["tns"] + g_wns * r["wns"]  # noqa: E731
    checked = 0
    for k in _fd_segments(d, 60, seed=4):
        cp, cm = base.copy(), base.copy()
        cp[k] += h
        cm[k] -= h
        rp, rm = oracle.smooth_sta(d, gamma, cp), oracle.smooth_sta(d, gamma, cm)
        if rp["sig"] != adj["sig"] or rm["sig"] != adj["sig"]:
            continue  # a table segment or slew winner changes inside [-h, h]
        fd = (J(rp) - J(rm)) / (2 * h)
        g = adj["grad_wire_cap"][k]
        assert abs(g - fd) <= 1e-5 * max(1.0, abs(fd)) + 1e-6, (k, g, fd)
        checked += 1
    assert checked >= 40


@pytest.mark.parametrize("g_tns,g_wns", [(1.0, 0.0), (0.0, 1.0)])
def test_resistance_gradient_matches_central_differences(small, g_tns, g_wns):
    """dJ/dR per segment against central differences of the FP64 objective
    with the segment's resistance moved by +-h (an FP64 override, so the step
    is exact)."""
    d, gamma = small, 5.0
    base = d.res_kohm.astype(np.float64)
    adj = oracle.smooth_adjoint(d, gamma, g_tns, g_wns, wire_res=base)
    J = lambda r: g_tns * r["tns"] + g_wns * r["wns"]  # noqa: E731
    assert np.all(adj["grad_wire_res"][d.net_node_ptr[:-1]] == 0.0)
    checked = 0
    for k in _fd_segments(d, 60, seed=9):
        h = 1e-3 * max(base[k], 1e-3)
        rp_, rm_ = base.copy(), base.copy()
        rp_[k] += h
        rm_[k] -= h
        rp, rm = oracle.smooth_sta(d, gamma, wire_res=rp_), oracle.smooth_sta(d, gamma, wire_res=rm_)
        if rp["sig"] != adj["sig"] or rm["sig"] != adj["sig"]:
            continue
        fd = (J(rp) - J(rm)) / (2 * h)
        g = adj["grad_wire_res"][k]
        assert abs(g - fd) <= 1e-5 * max(1.0, abs(fd)) + 1e-6, (k, g, fd)
        checked += 1
    assert checked >= 40
    assert np.abs(adj["grad_wire_res"]).max() > 0


def test_pin_load_gradient_by_differences(small):
    """grad_pin_load is the partial of the objective through each cell
    output's NLDM load only (not through the RC moments): central differences
    of the FP64 objective with that one load moved by +-h, on 60 seeded cell
    outputs."""
    d, gamma, h = small, 5.0, 1e-3
    adj = oracle.smooth_adjoint(d, gamma, 0.7, 0.3)
    J = lambda r: 0.7 * r["tns"] + 0.3 * r["wns"]  # noqa: E731
    net_of_drv = np.full(d.n_pins, -1)
    net_of_drv[d.net_driver] = np.arange(d.n_nets)
    outs = np.random.default_rng(5).choice(d.cell_out_pin, size=60, replace=False)
    checked = 0
    for p in outs:
        dl = np.zeros(d.n_nets)
        dl[net_of_drv[p]] = h
        rp, rm = oracle.smooth_sta(d, gamma, load_delta=dl), oracle.smooth_sta(d, gamma, load_delta=-dl)
        if rp["sig"] != adj["sig"] or rm["sig"] != adj["sig"]:
            continue
        fd = (J(rp) - J(rm)) / (2 * h)
        g = adj["grad_pin_load"][p]
        assert abs(g - fd) <= 1e-5 * max(1.0, abs(fd)) + 1e-6, (int(p), g, fd)
        checked += 1
    assert checked >= 40
    assert np.abs(adj["grad_pin_load"][outs]).max() > 0


def test_arc_delay_gradient_per_arc_by_differences(small):
    """grad_arc_delay per arc and view at gamma = 5 ps: central differences of
    the FP64 objective with one arc's delay in one view moved by +-h.  Late
    views on 40 seeded arcs; early views do not enter the objective, so both
    sides are zero there."""
    d, gamma, h = small, 5.0, 1e-3
    adj = oracle.smooth_adjoint(d, gamma, 1.0, 0.0)
    n_arcs = int(d.cell_in_ptr[-1])
    rng = np.random.default_rng(6)
    checked = nonzero = 0
    for k in rng.choice(n_arcs, size=40, replace=False):
        for v in (0, 2, 3):
            da = np.zeros((n_arcs, 4))
            da[k, v] = h
            rp, rm = oracle.smooth_sta(d, gamma, arc_delta=da), oracle.smooth_sta(d, gamma, arc_delta=-da)
            if rp["sig"] != adj["sig"] or rm["sig"] != adj["sig"]:
                continue
            fd = (rp["tns"] - rm["tns"]) / (2 * h)
            g = adj["grad_arc_delay"][k, v]
            if v == 0:
                assert g == 0.0 and fd == 0.0, (int(k), v, g, fd)
            else:
                assert abs(g - fd) <= 1e-5 * max(1.0, abs(fd)) + 1e-6, (int(k), v, g, fd)
                nonzero += abs(fd) > 1e-3
            checked += 1
    assert checked >= 100 and nonzero >= 10


def test_adjoint_on_the_1m_pin_design_at_200_segments():
    """The differentiable configuration as specified: the 1M-pin design, d TNS_g
    / d(wire C) of 200 RC segments drawn with seed 4, central differences with
    h = 1e-3 fF on the FP64 objective (segments whose step changes a table
    segment or slew winner are skipped and counted)."""
    from concurrent.futures import ThreadPoolExecutor
    d, gamma, h = synth.generate(synth.mid_config()), 5.0, 1e-3
    base = d.cap_ff.astype(np.float64)
    adj = oracle.smooth_adjoint(d, gamma, 1.0, 0.0, wire_cap=base)
    segs = _fd_segments(d, 200, seed=4)

    def fd(k):
        cp = base.copy()
        cp[k] += h
        rp = oracle.smooth_sta(d, gamma, cp)
        cp[k] = base[k] - h
        rm = oracle.smooth_sta(d, gamma, cp)
        if rp["sig"] != adj["sig"] or rm["sig"] != adj["sig"]:
            return None
        return (rp["tns"] - rm["tns"]) / (2 * h)

    with ThreadPoolExecutor(max_workers=8) as ex:  # the oracle call releases the GIL
        fds = list(ex.map(fd, segs))
    checked = 0
    for k, f in zip(segs, fds):
        if f is None:
            continue
        g = adj["grad_wire_cap"][k]
        assert abs(g - f) <= 1e-5 * max(1.0, abs(f)) + 1e-6, (int(k), g, f)
        checked += 1
    print(f"200 segments: {checked} checked, {200 - checked} skipped (a discrete choice moved)")
    assert checked >= 150


def test_hard_limit_arc_gradient_counts_violating_paths():
    """gamma -> 0 with slew-independent constant tables and no wire
    resistance: d TNS / d(arc delay) = -(number of violating endpoints whose
    critical path uses the arc), where an exact tie between m critical
    candidates splits the count 1/m each (the limit of the softmax)."""
    cfg = synth.SynthConfig(n_cells=40, n_levels=6, n_pi=4, n_po=4, fanout_mu=2.0, fanout_cap=4,
                            n_types=8, rat_ps=60.0, rat_early_ps=0.0, seed=77)
    d = synth.generate(cfg)
    rng = np.random.default_rng(3)
    for t in range(d.n_types):
        for k in range(4):
            d.tables[t, k] = np.float32(rng.uniform(2.0, 20.0))
    d.res_kohm[:] = 0.0
    adj = oracle.smooth_adjoint(d, 1e-3, 1.0, 0.0)
    g = adj["grad_arc_delay"][:, 2:]
    assert g.min() <= -1.0  # some arc lies on a violating critical path
    # count directly: push unit weights back from each violating endpoint
    hard = oracle.sta(d)
    at = hard["at"]
    W = np.zeros((d.n_pins, 2))
    for p in hard["ep_pin"]:
        sl = hard["slack"][p, 2:]
        if sl.min() < 0:
            tie = np.abs(sl - sl.min()) < 1e-9
            W[p] += tie / tie.sum()
    drv_of_sink = np.full(d.n_pins, -1)
    drv_of_sink[d.net_sink_pin] = np.repeat(d.net_driver, np.diff(d.net_sink_ptr))
    cell_of_out = np.full(d.n_pins, -1)
    cell_of_out[d.cell_out_pin] = np.arange(d.n_cells)
    count = np.zeros_like(g)
    for p in hard["level_order"][::-1]:
        if drv_of_sink[p] >= 0:
            W[drv_of_sink[p]] += W[p]
        elif cell_of_out[p] >= 0:
            c = cell_of_out[p]
            t, sense = d.cell_type[c], d.sense[d.cell_type[c]]
            for ro in (0, 1):
                if W[p, ro] == 0:
                    continue
                cands = []
                for k in range(d.cell_in_ptr[c], d.cell_in_ptr[c + 1]):
                    for ri in (0, 1):
                        if sense == 2 or (sense == 0) == (ri == ro):
                            z = at[d.cell_in_pin[k], 2 + ri] + float(d.tables[t, ro, 0, 0])
                            cands.append((z, k, ri))
                zmax = max(z for z, _, _ in cands)
                win = [(k, ri) for z, k, ri in cands if abs(z - zmax) < 1e-9]
                for k, ri in win:
                    w = W[p, ro] / len(win)
                    count[k, ro] -= w
                    W[d.cell_in_pin[k], ri] += w
    np.testing.assert_allclose(g, count, atol=1e-6)
