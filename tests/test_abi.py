"""C ABI checks that need no GPU: the library loads, exports every function
include/sta.h declares, and rejects malformed inputs during host validation
(before any device call) with the documented status codes."""
import ctypes
import os
import re

import numpy as np
import pytest

from designs import CIN, COUT, PI, PO, make_design, planar_table, single_segment_net
from paper_2511_11660_amd import sta as S
from paper_2511_11660_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _has_gpu():
    try:
        import torch
        return torch.cuda.device_count() > 0
    except Exception:
        return False


def test_exports_every_declared_function():
    hdr = open(os.path.join(ROOT, "include", "sta.h")).read()
    declared = set(re.findall(r"\b(sta_[a-z_]+)\s*\(", hdr))
    assert "sta_create" in declared and "sta_update_timing" in declared
    S.load()  # brings in the process's HIP runtime first
    lib = ctypes.CDLL(S.LIB_PATH)
    missing = [f for f in sorted(declared) if not hasattr(lib, f)]
    assert not missing, missing
    bound = {name for name, _, _ in S._SIGS}
    assert declared <= bound, declared - bound


def test_status_strings_and_defaults():
    assert S.sta_status_string(S.STA_E_CYCLE) == "STA_E_CYCLE"
    o = S.sta_options_default()
    assert o.mode == 0 and o.sort_endpoints == 1 and o.device == -1 and o.gamma_ps == 5.0


def _tiny():
    return synth.generate(synth.tiny_config())


def _create(d, **opts):
    keep = []
    g, rc, lib, cons = S.descriptors(d, keep)
    o = S.sta_options_default()
    for k, v in opts.items():
        setattr(o, k, v)
    return S.sta_create(g, rc, lib, cons, o)


def _expect(d, status, **opts):
    with pytest.raises(S.StaError) as e:
        _create(d, **opts)
    assert e.value.status == status, str(e.value)
    return str(e.value)


def test_rejects_bad_pin_kind():
    d = _tiny()
    d.pin_kind[5] = 7
    assert "kind" in _expect(d, S.STA_E_ARG)


def test_rejects_parent_not_less_than_child():
    d = _tiny()
    k = int(d.net_node_ptr[3]) + 2
    d.parent[k] = 5
    assert "parent" in _expect(d, S.STA_E_ARG)


def test_rejects_sink_node_outside_net():
    d = _tiny()
    d.sink_node[0] = 10_000
    _expect(d, S.STA_E_ARG)


def test_rejects_nan_and_negative_caps():
    d = _tiny()
    d.cap_ff[17] = np.nan
    _expect(d, S.STA_E_ARG)
    d = _tiny()
    d.res_kohm[17] = -1.0
    _expect(d, S.STA_E_ARG)


def test_rejects_non_increasing_axis():
    d = _tiny()
    d.slew_axis[2, 3] = d.slew_axis[2, 2]
    assert "axis" in _expect(d, S.STA_E_ARG)


def test_rejects_pin_on_two_nets():
    d = _tiny()
    d.net_sink_pin[1] = d.net_sink_pin[0]
    _expect(d, S.STA_E_ARG)


def test_rejects_wrong_input_count_for_type():
    d = _tiny()
    d.n_inputs[:] = 3
    assert "inputs" in _expect(d, S.STA_E_ARG)


def test_rejects_bad_mode_gamma_and_sizes():
    d = _tiny()
    _expect(d, S.STA_E_ARG, mode=5)
    _expect(d, S.STA_E_ARG, mode=1, gamma_ps=0.0)
    _expect(d, S.STA_E_ARG, mode=1, gamma_ps=float("nan"))
    _expect(d, S.STA_E_ARG, sched=7)
    d2 = _tiny()
    d2.nx = 9
    _expect(d2, S.STA_E_UNSUPPORTED)


def test_rejects_nan_constraint():
    d = _tiny()
    d.po_rat[0, 2] = np.inf
    _expect(d, S.STA_E_ARG)


def test_rejects_cell_without_inputs():
    kinds = [PI, COUT, CIN, COUT]
    cells = [(0, [], 1), (0, [2], 3)]
    nets = [single_segment_net(0, [2], 0.01, 1.0), single_segment_net(1, [], 0, 0),
            single_segment_net(3, [], 0, 0)]
    t = np.stack([np.stack([planar_table(5, 0.1, 1.0)] * 4)])
    d = make_design(kinds, cells, nets, n_inputs=[1], sense=[0], pin_cap=[1.0], tables=t)
    _expect(d, S.STA_E_ARG)


@pytest.mark.skipif(_has_gpu(), reason="checks the no-device error path")
def test_valid_design_without_device_reports_device_error():
    d = _tiny()
    msg = _expect(d, S.STA_E_DEVICE)
    assert msg


def test_null_context_calls_are_state_errors():
    with pytest.raises(S.StaError) as e:
        S.sta_update_timing(0)
    assert e.value.status == S.STA_E_STATE
    with pytest.raises(S.StaError) as e:
        S.sta_backward(0, 1.0, 0.0)
    assert e.value.status == S.STA_E_STATE
    with pytest.raises(S.StaError) as e:
        S.sta_update_timing_incremental(0, np.array([0], np.int32))
    assert e.value.status == S.STA_E_STATE


def test_reduced_order_delay_option_checks():
    d = _tiny()
    assert S.sta_options_default().delay_model == 0
    _expect(d, S.STA_E_ARG, delay_model=2)
    _expect(d, S.STA_E_UNSUPPORTED, delay_model=1, mode=1)


def test_estimate_rc_host_checks():
    d = synth.generate(synth.tiny_config(seed=5))
    x, y = synth.place(d, seed=2)
    for bad in ((-1.0, 0.0, 0.1, 0.1), (0.001, float("nan"), 0.1, 0.1), (0.001, 0.001, float("inf"), 0.1)):
        with pytest.raises(S.StaError) as e:
            S.estimate_rc(d, x, y, *bad)
        assert e.value.status == S.STA_E_ARG
    w = S.sta_wire_params(0.001, 0.001, 0.1, 0.1)
    g = S.sta_graph_desc()
    g.n_nets, g.n_pins, g.mem = 1, 1, 7
    assert S.load().sta_estimate_rc(ctypes.byref(g), None, None, ctypes.byref(w), None, None, None, None, None,
                                    S.STA_HOST, None) == S.STA_E_ARG
    if not _has_gpu():  # valid input: the first device call fails
        with pytest.raises(S.StaError) as e:
            S.estimate_rc(d, x, y, 0.001, 0.001, 0.1, 0.1)
        assert e.value.status == S.STA_E_DEVICE


def test_estimate_rc_noalloc_host_checks():
    """The allocation-free estimator takes device memory only and checks its
    arguments before any device call."""
    w = S.sta_wire_params(0.001, 0.001, 0.1, 0.1)
    g = S.sta_graph_desc()
    g.n_nets, g.n_pins, g.mem = 1, 1, S.STA_HOST
    assert S.load().sta_estimate_rc_noalloc(ctypes.byref(g), None, None, ctypes.byref(w), None, None, None, None,
                                            None, None) == S.STA_E_ARG
    assert b"device memory" in S.load().sta_last_error()
    g.mem = S.STA_DEVICE
    bad = S.sta_wire_params(0.001, -1.0, 0.1, 0.1)
    assert S.load().sta_estimate_rc_noalloc(ctypes.byref(g), None, None, ctypes.byref(bad), None, None, None, None,
                                            None, None) == S.STA_E_ARG


def _batch(designs, **opts):
    keep = []
    descs = [S.descriptors(d, keep) for d in designs]
    o = S.sta_options_default()
    for k, v in opts.items():
        setattr(o, k, v)
    lib = descs[0][2] if descs else S.sta_lib_desc()
    return S.sta_batch_create([x[0] for x in descs], [x[1] for x in descs], lib, [x[3] for x in descs], o)


def test_batch_validation_names_the_design():
    a, b = _tiny(), synth.generate(synth.tiny_config(seed=3))
    b.pin_kind[4] = 9
    with pytest.raises(S.StaError) as e:
        _batch([a, b])
    assert e.value.status == S.STA_E_ARG and "design 1:" in str(e.value), str(e.value)


def test_batch_rejects_smooth_mode_and_empty_batch():
    with pytest.raises(S.StaError) as e:
        _batch([_tiny(), _tiny()], mode=1)
    assert e.value.status == S.STA_E_UNSUPPORTED
    with pytest.raises(S.StaError) as e:
        _batch([])
    assert e.value.status == S.STA_E_ARG


def test_batch_null_context_calls_are_state_errors():
    for call in (lambda: S.sta_batch_report(0, 1), lambda: S.sta_autotune(0, 2),
                 lambda: S.sta_batch_offsets(0)):
        with pytest.raises(S.StaError) as e:
            call()
        assert e.value.status == S.STA_E_STATE
