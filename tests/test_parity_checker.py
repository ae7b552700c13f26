"""The parity checker itself, on the CPU: the oracle's own FP64 results rounded
to FP32 pass it, and planted mistakes (a shifted arrival, a wrong critical
fanin, a swapped endpoint pair, a level off by one) are caught."""
import numpy as np
import pytest

import oracle
from paper_2511_11660_amd import synth
from parity import compare_full


def _as_gpu(d, r):
    f = lambda a: np.asarray(a, np.float32)  # noqa: E731
    es = f(r["ep_slack"])
    order = np.stack([np.lexsort((r["ep_pin"], es[:, el])) for el in (0, 1)]).astype(np.int32)
    return {
        "levels": (r["level"].copy(), r["level_order"].copy()),
        "rc": (f(r["L_net"]), f(r["d_sink"]), f(r["q_sink"])),
        "timing": {"at": f(r["at"]), "slew": f(r["slew"]), "rat": f(r["rat"]), "crit": r["crit"].copy()},
        "slack": {"slack": f(r["slack"]), "ep_slack": es, "ep_order": order,
                  "wns": r["wns"].copy(), "tns": r["tns"].copy()},
        "ep_pin": r["ep_pin"].copy(),
    }


@pytest.fixture(scope="module")
def case():
    d = synth.generate(synth.mid_config(n_cells=5000, n_levels=20, seed=31))
    return d, oracle.sta(d)


def test_rounded_oracle_passes(case):
    d, r = case
    compare_full(d, r, _as_gpu(d, r))


def test_planted_arrival_shift_fails(case):
    d, r = case
    g = _as_gpu(d, r)
    p = int(d.cell_out_pin[100])
    g["timing"]["at"][p, 3] += 0.05
    with pytest.raises(AssertionError):
        compare_full(d, r, g)


def test_planted_rat_shift_fails(case):
    d, r = case
    g = _as_gpu(d, r)
    p = int(r["level_order"][10])
    g["timing"]["rat"][p, 2] -= 0.1
    with pytest.raises(AssertionError):
        compare_full(d, r, g)


def test_planted_wrong_crit_fails(case):
    d, r = case
    g = _as_gpu(d, r)
    # a 3-input cell whose late-rise winner is clearly separated from fanin 0
    for c in range(d.n_cells):
        a, b = d.cell_in_ptr[c], d.cell_in_ptr[c + 1]
        p = int(d.cell_out_pin[c])
        k = int(r["crit"][p, 2])
        if b - a >= 2 and k // 2 != 0 and d.sense[d.cell_type[c]] == 2:
            g["timing"]["crit"][p, 2] = 0 * 2 + (k % 2)
            break
    else:
        pytest.skip("no suitable cell")
    with pytest.raises(AssertionError):
        compare_full(d, r, g)


def test_planted_level_error_fails(case):
    d, r = case
    g = _as_gpu(d, r)
    g["levels"][0][5] += 1
    with pytest.raises(AssertionError):
        compare_full(d, r, g)


def test_planted_order_swap_fails(case):
    d, r = case
    g = _as_gpu(d, r)
    o = g["slack"]["ep_order"][1]
    es = r["ep_slack"][:, 1]
    # swap two endpoints whose slacks differ clearly
    i = int(np.argmax(np.abs(np.diff(es[o])) > 1.0))
    o[i], o[i + 1] = o[i + 1], o[i]
    with pytest.raises(AssertionError):
        compare_full(d, r, g)
