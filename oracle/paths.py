"""Top-k timing path report, FP64 CPU oracle.  TEST INFRASTRUCTURE ONLY (same
rule as the rest of ``oracle/``).

§III "Report options" of the paper lists top-k path reports controlled by k, a
per-endpoint report limit and a slack-less-than threshold, returned as flattened
CSR path-pin arrays with slacks.  The definitions used here are the textbook
graph-based ones on the timing graph of ``oracle.sta``:

* a path is a sequence of (pin, transition) from a primary input to an
  endpoint, following net arcs (driver -> sink, transition kept) and cell arcs
  (input -> output, transitions as the type's unateness allows);
* its arrival is the startpoint arrival plus the arc delays, each arc delay
  being the one the graph-based propagation uses (net arc: the sink's Elmore
  delay; cell arc: the NLDM delay at the input pin's propagated slew and the
  output net's load);
* late slack = endpoint RAT - arrival; early slack = arrival - endpoint RAT
  (both per endpoint transition);
* the report holds, over all endpoints, the paths of smallest slack with at
  most `per_endpoint` per endpoint, only those with slack < `slack_below`, and
  at most `k` in all, in ascending slack.

The enumeration is a plain best-first search over partial paths grown backward
from the endpoints: a partial path ending (towards the inputs) at node v has
key = (best slack of any path through it) = endpoint slack + sum of the
deviations taken so far, where moving from v to a predecessor u over arc e adds
dev = AT(v) - (AT(u) + delay(e)) (late) or (AT(u) + delay(e)) - AT(v) (early),
both >= 0.  Keys never decrease along a path, so complete paths come off the
heap in ascending slack.  ``all_paths`` enumerates every path exhaustively
(small designs only) to pin this.
"""
from __future__ import annotations

import heapq

import numpy as np

from . import nldm, sta as _sta

PI, CIN, COUT, PO = 0, 1, 2, 3


class _Graph:
    """Predecessor arcs of every (pin, transition) with their delays per
    early/late, from a full oracle timing result."""

    def __init__(self, d, r):
        self.d, self.r = d, r
        self.kind = np.asarray(d.pin_kind)
        self.drv_of_sink = np.full(d.n_pins, -1, np.int64)
        self.sink_idx = np.full(d.n_pins, -1, np.int64)
        for n in range(d.n_nets):
            for s in range(d.net_sink_ptr[n], d.net_sink_ptr[n + 1]):
                p = int(d.net_sink_pin[s])
                self.drv_of_sink[p] = int(d.net_driver[n])
                self.sink_idx[p] = s
        self.cell_of_out = np.full(d.n_pins, -1, np.int64)
        self.cell_of_out[np.asarray(d.cell_out_pin)] = np.arange(d.n_cells)
        self.net_of_drv = np.full(d.n_pins, -1, np.int64)
        self.net_of_drv[np.asarray(d.net_driver)] = np.arange(d.n_nets)

    def preds(self, p, rf, el):
        """[(u, rf_u, delay)] of node (p, rf) in early (el=0) / late (el=1)."""
        d, r = self.d, self.r
        k = self.kind[p]
        if k == CIN or k == PO:
            return [(int(self.drv_of_sink[p]), rf, float(r["d_sink"][self.sink_idx[p]]))]
        if k == COUT:
            c = int(self.cell_of_out[p])
            t = int(d.cell_type[c])
            sense = int(d.sense[t])
            load = float(r["L_net"][self.net_of_drv[p]])
            out = []
            for f in range(d.cell_in_ptr[c], d.cell_in_ptr[c + 1]):
                i = int(d.cell_in_pin[f])
                for ri in (0, 1):
                    if not (sense == 2 or (sense == 0 and ri == rf) or (sense == 1 and ri != rf)):
                        continue
                    x = float(r["slew"][i, el * 2 + ri])
                    dl = float(nldm(d.slew_axis[t], d.load_axis[t], d.tables[t, rf], x, load))
                    out.append((i, ri, dl))
            return out
        return []  # primary input


def _ep_views(r, el):
    """(endpoint index, pin, rf, RAT) of every constrained endpoint view."""
    out = []
    for e, p in enumerate(r["ep_pin"]):
        for rf in (0, 1):
            rat = float(r["rat"][p, el * 2 + rf])
            if np.isfinite(rat):
                out.append((e, int(p), rf, rat))
    return out


def _finish(found, k, per_endpoint):
    found.sort(key=lambda t: (t[0], t[1]))
    out, per = [], {}
    for slack, e, path in found:
        if per.get(e, 0) >= per_endpoint:
            continue
        per[e] = per.get(e, 0) + 1
        out.append({"slack": slack, "endpoint": e, "pins": [p for p, _ in path], "rf": [t for _, t in path]})
        if len(out) >= k:
            break
    return out


def top_paths(d, k, per_endpoint=1, slack_below=np.inf, el=1, r=None):
    """The path report defined in the module docstring, by best-first search.
    Returns a list of dicts (slack, endpoint index, pins and transitions from
    startpoint to endpoint) in ascending slack."""
    r = _sta(d) if r is None else r
    g = _Graph(d, r)
    at = r["at"]
    heap, seq = [], 0
    for e, p, rf, rat in _ep_views(r, el):
        a = float(at[p, el * 2 + rf])
        key = rat - a if el == 1 else a - rat
        heapq.heappush(heap, (key, seq, e, ((p, rf),)))
        seq += 1
    found, per = [], {}
    while heap and len(found) < k:
        key, _, e, path = heapq.heappop(heap)
        if key >= slack_below:
            break
        if per.get(e, 0) >= per_endpoint:
            continue
        p, rf = path[0]
        pr = g.preds(p, rf, el)
        if not pr:  # reached a primary input: a complete path
            per[e] = per.get(e, 0) + 1
            found.append((key, e, path))
            continue
        av = float(at[p, el * 2 + rf])
        for u, ru, dl in pr:
            au = float(at[u, el * 2 + ru])
            dev = av - (au + dl) if el == 1 else (au + dl) - av
            heapq.heappush(heap, (key + max(dev, 0.0), seq, e, ((u, ru),) + path))
            seq += 1
    return _finish(found, k, per_endpoint)


def all_paths(d, el=1, r=None):
    """Every path to every constrained endpoint view with its slack, by
    exhaustive backward enumeration, arrivals summed along each path (small
    designs only).  Returns [(slack, endpoint index, path)], unsorted."""
    r = _sta(d) if r is None else r
    g = _Graph(d, r)
    out = []

    def walk(p, rf, acc, path, e, rat):
        pr = g.preds(p, rf, el)
        if not pr:
            arrival = float(r["at"][p, el * 2 + rf]) + acc  # startpoint arrival + arc delays
            out.append(((rat - arrival) if el == 1 else (arrival - rat), e, path))
            return
        for u, ru, dl in pr:
            walk(u, ru, acc + dl, ((u, ru),) + path, e, rat)

    for e, p, rf, rat in _ep_views(r, el):
        walk(p, rf, 0.0, ((p, rf),), e, rat)
    return out


def brute_top_paths(d, k, per_endpoint=1, slack_below=np.inf, el=1, r=None):
    """The same report from ``all_paths`` (the definition, summed directly)."""
    found = [t for t in all_paths(d, el, r) if t[0] < slack_below]
    return _finish(found, k, per_endpoint)
