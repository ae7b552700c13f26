"""Element-wise comparison of the HIP path against the FP64 oracle.

Tolerance (FP32 GPU vs FP64 oracle): |g - o| <= max(1e-3 ps, 1e-5 S) where S
is the magnitude the value is computed from.  Arrival and slew: the largest
finite |AT| (resp. |slew|) on the pin's fanin cone; for non-negative arrivals
this is |AT| itself, and a slew extrapolated from a huge input slew (an
unbuffered 9k-sink net gives 86 ns, 580x past the table) carries the FP32
rounding of that input.  Required time is a chain of subtractions from the endpoint
required times down to the pin, so S is the largest finite |RAT| on the pin's
fanout cone: a RAT near zero derived from a 4500 ps endpoint carries FP32
rounding of 4500 ps operands.  Slack: the larger of the two.  Scales are per
pin and per early/late.  Infinities must match exactly.  Levels and the
level order are integers: exact.  Critical fanin and endpoint order are exact
except inside ties: a GPU choice that differs from the oracle's is accepted iff
the oracle's FP64 value for the GPU's choice is within tolerance of the optimum.
"""
from __future__ import annotations

import numpy as np

import oracle

REL, ABS = 1e-5, 1e-3


def tol(ref):
    return np.maximum(ABS, REL * np.abs(ref))


def check_close(name, g, o, scale=None):
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    assert g.shape == o.shape, (name, g.shape, o.shape)
    inf_o = ~np.isfinite(o)
    bad_inf = inf_o & (g != o)
    assert not bad_inf.any(), f"{name}: infinities differ at {np.argwhere(bad_inf)[:5].tolist()}"
    t = tol(o if scale is None else scale)
    with np.errstate(invalid="ignore"):
        err = np.where(inf_o, 0.0, np.abs(g - o))
    bad = err > t
    if bad.any():
        idx = np.argwhere(bad)[:5].tolist()
        raise AssertionError(f"{name}: {int(bad.sum())} of {g.size} outside tolerance; first {idx}; "
                             f"max err {err.max():.3e}")
    return float(err.max()) if err.size else 0.0


def crit_check(d, r, crit_g, at_scale):
    """Critical fanin per cell-output view: exact, or a near-tie (returns the
    number of near-ties accepted)."""
    cell_of_out = np.full(d.n_pins, -1, np.int64)
    cell_of_out[d.cell_out_pin] = np.arange(d.n_cells)
    net_of_drv = np.full(d.n_pins, -1, np.int64)
    net_of_drv[d.net_driver] = np.arange(d.n_nets)
    crit_o = r["crit"]
    diff = np.argwhere(crit_g != crit_o)
    ties = 0
    for p, v in diff:
        p, v = int(p), int(v)
        assert cell_of_out[p] >= 0, f"crit differs on non-cell-output pin {p}"
        c = cell_of_out[p]
        k = int(crit_g[p, v])
        assert k >= 0, f"crit missing at pin {p} view {v}"
        el, ro, ri = v // 2, v % 2, k % 2
        pin_in = int(d.cell_in_pin[d.cell_in_ptr[c] + k // 2])
        t = int(d.cell_type[c])
        sense = int(d.sense[t])
        ok_map = sense == 2 or (sense == 0 and ri == ro) or (sense == 1 and ri != ro)
        assert ok_map, f"crit at pin {p} view {v} names an arc the unateness forbids"
        load = r["L_net"][net_of_drv[p]]
        x = r["slew"][pin_in, el * 2 + ri]
        cand = r["at"][pin_in, el * 2 + ri] + oracle.nldm(d.slew_axis[t], d.load_axis[t],
                                                          d.tables[t, ro], x, load)
        best = r["at"][p, v]
        assert abs(cand - best) <= tol(at_scale[p, v]), \
            f"crit at pin {p} view {v}: GPU picked {k} (value {cand}), oracle {crit_o[p, v]} ({best})"
        ties += 1
    return ties


def order_check(ep_pin, ep_slack_o, ep_slack_g, order_o, order_g, scale):
    """Endpoint order: a permutation, sorted by (GPU slack, pin id) exactly,
    and position-wise equal to the oracle's order up to tolerance ties."""
    ne = len(ep_pin)
    ties = 0
    for el in (0, 1):
        g = order_g[el]
        assert np.array_equal(np.sort(g), np.arange(ne)), "endpoint order is not a permutation"
        sv, pv = ep_slack_g[g, el], ep_pin[g]
        asc = (sv[1:] > sv[:-1]) | ((sv[1:] == sv[:-1]) & (pv[1:] > pv[:-1]))
        assert asc.all(), "endpoint order not ascending in (slack, pin id)"
        o = order_o[el]
        neq = g != o
        if neq.any():
            vg = ep_slack_o[g, el]
            vo = ep_slack_o[o, el]
            t = tol(scale[o, el])
            bad = neq & (np.abs(vg - vo) > t)
            assert not bad.any(), f"endpoint order differs beyond ties at {np.argwhere(bad)[:5].tolist()}"
            ties += int(neq.sum())
    return ties


def _levels(r):
    order = r["level_order"]
    lv = r["level"][order]
    bounds = np.searchsorted(lv, np.arange(lv.max() + 2))
    return order, bounds


def _absfin(v):
    a = np.where(np.isfinite(v), np.abs(v), 0.0)
    return np.stack([a[:, :2].max(1), a[:, 2:].max(1)], 1)


def _segmax(vals, members, starts, ends):
    """max over vals[members[starts[i]:ends[i]]] per segment (segments non-empty)."""
    lens = ends - starts
    off = np.concatenate([[0], np.cumsum(lens)[:-1]])
    idx = np.repeat(starts - off, lens) + np.arange(lens.sum())
    return np.maximum.reduceat(vals[members[idx]], off, axis=0)


def magnitude_scales(d, r):
    """(fanin-cone max |AT|, fanout-cone max |RAT|, fanin-cone max |slew|) per
    pin and early/late."""
    NP = d.n_pins
    order, bounds = _levels(r)
    cin_out = np.full(NP, -1, np.int64)
    nin = np.diff(d.cell_in_ptr)
    cin_out[d.cell_in_pin] = np.repeat(d.cell_out_pin, nin)
    net_of_drv = np.full(NP, -1, np.int64)
    net_of_drv[d.net_driver] = np.arange(d.n_nets)
    drv_of_sink = np.full(NP, -1, np.int64)
    drv_of_sink[d.net_sink_pin] = np.repeat(d.net_driver, np.diff(d.net_sink_ptr))
    cell_of_out = np.full(NP, -1, np.int64)
    cell_of_out[d.cell_out_pin] = np.arange(d.n_cells)
    U = _absfin(r["at"])
    M = _absfin(r["rat"])
    S = _absfin(r["slew"])
    nl = len(bounds) - 1
    for lv in range(nl):  # fanin cone, ascending levels
        pins = order[bounds[lv]:bounds[lv + 1]]
        sk = pins[drv_of_sink[pins] >= 0]
        U[sk] = np.maximum(U[sk], U[drv_of_sink[sk]])
        S[sk] = np.maximum(S[sk], S[drv_of_sink[sk]])
        co = pins[cell_of_out[pins] >= 0]
        if len(co):
            c = cell_of_out[co]
            U[co] = np.maximum(U[co], _segmax(U, d.cell_in_pin, d.cell_in_ptr[c], d.cell_in_ptr[c + 1]))
            S[co] = np.maximum(S[co], _segmax(S, d.cell_in_pin, d.cell_in_ptr[c], d.cell_in_ptr[c + 1]))
    for lv in range(nl - 1, -1, -1):  # fanout cone, descending levels
        pins = order[bounds[lv]:bounds[lv + 1]]
        ci = pins[cin_out[pins] >= 0]
        M[ci] = np.maximum(M[ci], M[cin_out[ci]])
        dr = pins[net_of_drv[pins] >= 0]
        if len(dr):
            n = net_of_drv[dr]
            a, b = d.net_sink_ptr[n], d.net_sink_ptr[n + 1]
            ne = b > a
            if ne.any():
                M[dr[ne]] = np.maximum(M[dr[ne]], _segmax(M, d.net_sink_pin, a[ne], b[ne]))
    return U, M, S


def _view_scale(S):
    return np.repeat(S, 2, axis=1)


def compare_full(d, r, gpu, *, check_order=True, scales=None):
    """Compares a full GPU run (dict from STA.timing/slack/levels/rc) with the
    oracle result r on design d.  Returns a dict of statistics.  scales: the
    magnitude_scales(d, r) triple, when the caller compares several runs
    against one oracle result."""
    stats = {}
    lv, lo = gpu["levels"]
    np.testing.assert_array_equal(lv, r["level"])
    np.testing.assert_array_equal(lo, r["level_order"])
    L, dd, q = gpu["rc"]
    stats["L_net"] = check_close("L_net", L, r["L_net"])
    stats["d"] = check_close("sink delay", dd, r["d_sink"])
    # q = 2 m2 - d^2 cancels; its FP32 error scales with d * (largest d on the net)
    fo = np.diff(d.net_sink_ptr)
    ne = fo > 0
    net_dmax = np.zeros(d.n_nets)
    if ne.any():
        net_dmax[ne] = np.maximum.reduceat(r["d_sink"], d.net_sink_ptr[:-1][ne])
    dmax = np.repeat(net_dmax, fo)
    qt = 1e-5 * np.abs(r["q_sink"]) + 1e-5 * r["d_sink"] * dmax + 1e-9
    qerr = np.abs(q - r["q_sink"])
    assert (qerr <= qt).all(), f"sink spread outside tolerance at {np.argwhere(qerr > qt)[:5].ravel().tolist()}"
    t = gpu["timing"]
    U, M, S = magnitude_scales(d, r) if scales is None else scales
    Uv, Mv = _view_scale(U), _view_scale(M)
    stats["at"] = check_close("AT", t["at"], r["at"], Uv)
    stats["slew"] = check_close("slew", t["slew"], r["slew"], _view_scale(S))
    stats["rat"] = check_close("RAT", t["rat"], r["rat"], Mv)
    s = gpu["slack"]
    scale = np.maximum(Uv, Mv)
    stats["slack"] = check_close("slack", s["slack"], r["slack"], scale)
    stats["crit_ties"] = crit_check(d, r, t["crit"], Uv)
    np.testing.assert_array_equal(gpu["ep_pin"], r["ep_pin"])
    ep_scale = np.stack([scale[r["ep_pin"], 0:2].max(1), scale[r["ep_pin"], 2:4].max(1)], 1)
    check_close("endpoint slack", s["ep_slack"], r["ep_slack"], ep_scale)
    for el in (0, 1):
        viol = r["ep_slack"][:, el] < tol(ep_scale[:, el])
        tns_tol = tol(ep_scale[viol, el]).sum() + 1e-6
        assert abs(s["tns"][el] - r["tns"][el]) <= tns_tol, (el, s["tns"][el], r["tns"][el], tns_tol)
        wi = int(np.argmin(r["ep_slack"][:, el])) if len(r["ep_slack"]) else 0
        wt = tol(ep_scale[wi, el]) if len(r["ep_slack"]) else ABS
        assert abs(s["wns"][el] - r["wns"][el]) <= wt, (el, s["wns"][el], r["wns"][el])
    if check_order:
        stats["order_ties"] = order_check(r["ep_pin"], r["ep_slack"], s["ep_slack"], r["ep_order"],
                                          s["ep_order"], ep_scale)
    return stats


def assert_bitwise_equal(a, b, where=""):
    """Two run_gpu dicts hold bit-identical results (levels, RC, timing,
    critical fanins, slacks, WNS/TNS and endpoint order)."""
    for x, y, k in zip(a["levels"], b["levels"], ("level", "level_order")):
        assert np.array_equal(x, y), (where, k)
    for x, y, k in zip(a["rc"], b["rc"], ("L_net", "d", "q")):
        assert np.array_equal(x.view(np.uint32), y.view(np.uint32)), (where, k)
    for k, v in a["timing"].items():
        w = b["timing"][k]
        assert v.dtype == w.dtype and np.array_equal(v.view(np.uint8), w.view(np.uint8)), (where, k)
    for k in ("slack", "ep_slack", "ep_order", "wns", "tns"):
        v, w = np.asarray(a["slack"][k]), np.asarray(b["slack"][k])
        assert v.dtype == w.dtype and np.array_equal(v.view(np.uint8), w.view(np.uint8)), (where, k)
    assert np.array_equal(a["ep_pin"], b["ep_pin"]), (where, "ep_pin")


def run_gpu(sta_obj):
    return {
        "levels": sta_obj.levels(),
        "rc": sta_obj.rc(),
        "timing": sta_obj.timing(),
        "slack": sta_obj.slack(),
        "ep_pin": sta_obj.endpoints(),
    }
