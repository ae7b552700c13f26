"""Pins of the path-report oracle (oracle/paths.py) on the CPU: its best-first
search against exhaustive enumeration with arrivals summed along each path, the
one-path-per-endpoint case against the endpoint slacks of the timing oracle,
and the validity of every reported path."""
import numpy as np
import pytest

import oracle
from designs import CIN, COUT, PI, PO, make_design, planar_table, single_segment_net
from oracle import paths as P


def small_dag(seed, n_pi=5, levels=3, per_level=4, n_inputs=(1, 2, 3, 2)):
    """A small random timing DAG (every cell of 1-3 inputs, or of the four
    types' n_inputs, drawn from earlier levels, multi-sink star nets, mixed
    unateness) whose paths can all be enumerated."""
    rng = np.random.default_rng(seed)
    kinds, cells, sinks_of = [], [], {}

    def pin(k):
        kinds.append(k)
        return len(kinds) - 1

    pis = [pin(PI) for _ in range(n_pi)]
    for p in pis:
        sinks_of[p] = []
    avail, prev = list(pis), list(pis)
    n_inputs = list(n_inputs)
    for _ in range(levels):
        outs = []
        for _ in range(per_level):
            t = int(rng.integers(0, 4))
            srcs = [int(rng.choice(prev))] + [int(rng.choice(avail)) for _ in range(n_inputs[t] - 1)]
            ins = []
            for src in srcs:
                ci = pin(CIN)
                sinks_of[src].append(ci)
                ins.append(ci)
            o = pin(COUT)
            sinks_of[o] = []
            cells.append((t, ins, o))
            outs.append(o)
        avail += outs
        prev = outs
    for o in prev:
        sinks_of[o].append(pin(PO))
    nets = [single_segment_net(drv, sk, float(rng.uniform(0.01, 0.05)), float(rng.uniform(0.5, 2.0)))
            for drv, sk in sinks_of.items()]
    tables = np.stack([np.stack([planar_table(6 + 2 * t, 0.1 + 0.02 * t, 1.0, 0.001 * t),
                                 planar_table(7 + t, 0.12, 1.2),
                                 planar_table(3, 0.05, 2.0 + 0.1 * t),
                                 planar_table(4, 0.06, 1.8)]) for t in range(4)])
    return make_design(kinds, cells, nets, n_inputs=n_inputs, sense=[1, 0, 2, 1],
                       pin_cap=[1.0, 1.2, 0.9, 1.5], tables=tables, po_rat=60.0, rat_early=25.0,
                       pi_at=0.0, pi_slew=20.0, dangling_policy=1)


def _connected(d, path):
    """Every step of a reported path is an arc of the timing graph."""
    drv = {int(d.net_sink_pin[s]): int(d.net_driver[n]) for n in range(d.n_nets)
           for s in range(d.net_sink_ptr[n], d.net_sink_ptr[n + 1])}
    cell_in = {int(d.cell_out_pin[c]): (set(int(p) for p in d.cell_in_pin[d.cell_in_ptr[c]:d.cell_in_ptr[c + 1]]),
                                        int(d.sense[d.cell_type[c]])) for c in range(d.n_cells)}
    pins, rf = path["pins"], path["rf"]
    assert d.pin_kind[pins[0]] == PI
    for a, b, ra, rb in zip(pins[:-1], pins[1:], rf[:-1], rf[1:]):
        if b in drv:
            assert drv[b] == a and ra == rb
        else:
            ins, sense = cell_in[b]
            assert a in ins
            assert sense == 2 or (sense == 0 and ra == rb) or (sense == 1 and ra != rb)


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
@pytest.mark.parametrize("el", [0, 1])
def test_best_first_matches_exhaustive_enumeration(seed, el):
    d = small_dag(seed)
    r = oracle.sta(d)
    for k, per_ep, thr in [(10, 1, np.inf), (25, 3, np.inf), (1000, 1000, np.inf), (40, 5, 5.0)]:
        got = P.top_paths(d, k, per_ep, thr, el, r)
        ref = P.brute_top_paths(d, k, per_ep, thr, el, r)
        assert len(got) == len(ref)
        np.testing.assert_allclose([g["slack"] for g in got], [x["slack"] for x in ref], rtol=0, atol=1e-9)
        for g in got:
            _connected(d, g)
            assert g["slack"] < thr


@pytest.mark.parametrize("el", [0, 1])
def test_one_path_per_endpoint_is_the_endpoint_slack(el):
    d = small_dag(7, n_pi=6, levels=4, per_level=5)
    r = oracle.sta(d)
    got = P.top_paths(d, 10_000, 1, np.inf, el, r)
    ep_slack = r["ep_slack"][:, el]
    finite = np.isfinite(ep_slack)
    assert len(got) == int(finite.sum())
    np.testing.assert_allclose(sorted(g["slack"] for g in got), np.sort(ep_slack[finite]), atol=1e-9)
    # the worst path's slack is constant along it (graph-based critical path)
    worst = got[0]
    pins, rf = worst["pins"], worst["rf"]
    vi = [el * 2 + t for t in rf]
    s = [r["slack"][p, v] for p, v in zip(pins, vi)]
    np.testing.assert_allclose(s, s[-1], atol=1e-9)


def test_all_paths_count_on_a_hand_counted_design():
    """PI0 -> INV -> NAND2(other input PI1) -> BUF -> PO: two startpoints, one
    path from each per endpoint transition (inverting stages fix the input
    transition), so 2 x 2 paths for the late report."""
    kinds = [PI, PI, CIN, COUT, CIN, CIN, COUT, CIN, COUT, PO]
    cells = [(0, [2], 3), (1, [4, 5], 6), (2, [7], 8)]
    nets = [single_segment_net(0, [2], 0.02, 1.0), single_segment_net(1, [5], 0.02, 1.0),
            single_segment_net(3, [4], 0.02, 1.0), single_segment_net(6, [7], 0.02, 1.0),
            single_segment_net(8, [9], 0.02, 1.0)]
    t = planar_table(10, 0.1, 1.0)
    tables = np.stack([np.stack([t, t, planar_table(3, 0.05, 2.0), planar_table(3, 0.05, 2.0)])] * 3)
    d = make_design(kinds, cells, nets, n_inputs=[1, 2, 1], sense=[1, 1, 0], pin_cap=[1.0] * 3,
                    tables=tables, po_rat=500.0)
    allp = P.all_paths(d, el=1)
    assert len(allp) == 4
    starts = sorted(path[0][0] for _, _, path in allp)
    assert starts == [0, 0, 1, 1]
