"""GPU top-k path report against the FP64 path oracle: same slacks in the same
order (within the FP32 tolerance), the same pin sequences wherever slacks are
not tied, and every reported path a valid timing path whose FP64 slack,
summed along it with the oracle's arc delays, matches."""
import numpy as np
import pytest

import oracle
from oracle import paths as P
from paper_2511_11660_amd import synth
from paper_2511_11660_amd.sta import STA, STA_SCHED_PER_LEVEL, STA_SCHED_PERSISTENT
from designs import PI
from test_oracle_paths import _connected, small_dag

pytestmark = pytest.mark.gpu


def _scale(r):
    a = r["at"][np.isfinite(r["at"])]
    rt = r["rat"][np.isfinite(r["rat"])]
    return max(float(np.abs(a).max()), float(np.abs(rt).max()) if rt.size else 0.0)


def _fp64_slack(g, r, path, el):
    """Slack of a reported path from the oracle's FP64 arc delays."""
    acc = float(r["at"][path["pins"][0], el * 2 + path["rf"][0]])
    for a, b, ra, rb in zip(path["pins"][:-1], path["pins"][1:], path["rf"][:-1], path["rf"][1:]):
        for u, ru, dl in g.preds(b, rb, el):
            if u == a and ru == ra:
                acc += dl
                break
        else:
            raise AssertionError("not an arc")
    rat = float(r["rat"][path["pins"][-1], el * 2 + path["rf"][-1]])
    return rat - acc if el == 1 else acc - rat


def _compare(d, got, ref, r, el, thr, k, m):
    tol = max(1e-3, 1e-5 * _scale(r))
    gs = np.array([p["slack"] for p in got])
    rs = np.array([p["slack"] for p in ref])
    # paths within tolerance of the threshold may fall on either side
    near = lambda s: np.isfinite(thr) and abs(s - thr) <= tol
    if len(gs) != len(rs):
        extra = gs[len(rs):] if len(gs) > len(rs) else rs[len(gs):]
        assert all(near(s) for s in extra), (len(gs), len(rs))
    n = min(len(gs), len(rs))
    assert np.all(np.abs(gs[:n] - rs[:n]) <= tol), np.abs(gs[:n] - rs[:n]).max()
    g = P._Graph(d, r)
    # every oracle path of each endpoint near the reported slacks (a tie may
    # hide behind the per-endpoint limit): a GPU path must be one of the
    # oracle's paths of its endpoint within tolerance of its slack
    wide = P.top_paths(d, 4 * k + 16, m + 4, thr + 2 * tol if np.isfinite(thr) else thr, el, r)
    by_ep = {}
    for p in wide:
        by_ep.setdefault(p["endpoint"], []).append(p)
    for i in range(n):
        _connected(d, got[i])
        assert abs(_fp64_slack(g, r, got[i], el) - gs[i]) <= tol
        cands = [p for p in by_ep.get(got[i]["endpoint"], []) if abs(p["slack"] - gs[i]) <= 2 * tol]
        assert any(p["pins"] == got[i]["pins"] and p["rf"] == got[i]["rf"] for p in cands), i


@pytest.mark.parametrize("sched", [STA_SCHED_PERSISTENT, STA_SCHED_PER_LEVEL])
@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_paths_small_dags(seed, sched):
    d = small_dag(seed)
    r = oracle.sta(d)
    s = STA(d, sched=sched)
    s.update()
    for el in (0, 1):
        for k, m, thr in [(10, 1, np.inf), (25, 3, np.inf), (500, 64, np.inf), (40, 5, 5.0)]:
            got = s.paths(k, m, thr, el)
            ref = P.top_paths(d, k, m, thr, el, r)
            _compare(d, got, ref, r, el, thr, k, m)
    s.close()


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_paths_five_input_cells(seed):
    """A library type of five inputs: the walk reads each cell's fanins from
    the CSR lists instead of the inline four."""
    d = small_dag(seed, n_inputs=(1, 2, 5, 2))
    assert max(d.n_inputs) == 5
    r = oracle.sta(d)
    s = STA(d)
    s.update()
    for el in (0, 1):
        for k, m, thr in [(25, 3, np.inf), (500, 64, np.inf), (40, 5, 5.0)]:
            got = s.paths(k, m, thr, el)
            ref = P.top_paths(d, k, m, thr, el, r)
            _compare(d, got, ref, r, el, thr, k, m)
    s.close()


def test_paths_queues_in_global_memory(monkeypatch):
    """The endpoint queues in global memory (taken when they and the library
    do not fit in LDS) give the same report as the LDS queues."""
    d = synth.generate(synth.mid_config(seed=19, n_cells=30_000, n_levels=25))
    s = STA(d)
    s.update()
    cases = [(300, 8, np.inf, 1), (200, 64, np.inf, 0), (100, 3, 0.0, 1)]
    lds = [s.paths(*c) for c in cases]
    monkeypatch.setenv("STA_PATH_QUEUES_GLOBAL", "1")
    glob = [s.paths(*c) for c in cases]
    s.close()
    for a, b in zip(lds, glob):
        assert len(a) == len(b) and len(a) > 0
        for p, q in zip(a, b):
            assert p["endpoint"] == q["endpoint"] and p["slack"] == q["slack"]
            assert list(p["pins"]) == list(q["pins"]) and list(p["rf"]) == list(q["rf"])


def test_paths_tiny_design():
    d = synth.generate(synth.tiny_config(seed=5, dangling_policy=1))
    r = oracle.sta(d)
    s = STA(d)
    s.update()
    for el, k, m, thr in [(1, 200, 4, np.inf), (1, 500, 1, 0.0), (0, 100, 8, np.inf)]:
        got = s.paths(k, m, thr, el)
        ref = P.top_paths(d, k, m, thr, el, r)
        _compare(d, got, ref, r, el, thr, k, m)
    s.close()


def test_paths_mid_design_violators():
    d = synth.generate(synth.mid_config(seed=19, n_cells=30_000, n_levels=25))
    r = oracle.sta(d)
    s = STA(d)
    s.update()
    got = s.paths(300, 2, 0.0, 1)
    ref = P.top_paths(d, 300, 2, 0.0, 1, r)
    _compare(d, got, ref, r, 1, 0.0, 300, 2)
    s.close()


def test_paths_empty_and_threshold_edges():
    d = small_dag(2)
    s = STA(d)
    s.update()
    assert s.paths(10, 1, -1e9, 1) == []
    one = s.paths(1, 1, np.inf, 1)
    assert len(one) == 1
    s.close()


def test_paths_10m_worst_late():
    """The benchmark's 10M-pin design: the 200 worst late paths (at most 2 per
    endpoint) against the oracle's, rank by rank in slack, and every reported
    path a timing path whose FP64 slack, summed with the oracle's arc delays,
    matches."""
    d = synth.generate(synth.large_config())
    print(f"[paths] 10M design: {d.n_pins} pins", flush=True)
    s = STA(d)
    s.update()
    got = s.paths(200, 2, np.inf, 1)
    s.close()
    print("[paths] GPU report done", flush=True)
    r = oracle.sta(d)
    print("[paths] oracle timing done", flush=True)
    ref = P.top_paths(d, 200, 2, np.inf, 1, r)
    print("[paths] oracle paths done", flush=True)
    tol = max(1e-3, 1e-5 * _scale(r))
    gs = np.array([p["slack"] for p in got])
    rs = np.array([p["slack"] for p in ref])
    assert len(gs) == len(rs) == 200
    assert np.all(np.abs(gs - rs) <= tol), np.abs(gs - rs).max()
    g = P._Graph(d, r)
    print("[paths] oracle graph done", flush=True)
    kind = np.asarray(d.pin_kind)
    for p in got:  # (_fp64_slack asserts that every step is an arc of the graph)
        assert kind[p["pins"][0]] == PI  # a path starts at a primary input
        assert abs(_fp64_slack(g, r, p, 1) - p["slack"]) <= tol
