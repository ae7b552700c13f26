"""The allocation-free RC estimator (sta_estimate_rc_noalloc, fixed device
scratch) against the allocating one (sta_estimate_rc, per-call scratch) on the
same device inputs, through the C ABI: every output bit for bit, on two calls
in a row (the second smaller, so stale list entries or check words of the
first call would show), with nets in all three tiers (8-lane group, wave,
block), and the error beyond the fixed scratch."""
from types import SimpleNamespace

import numpy as np
import pytest

from paper_2511_11660_amd.sta import (STA_DEVICE, STA_E_UNSUPPORTED, StaError, sta_estimate_rc,
                                      sta_estimate_rc_noalloc, sta_graph_desc, sta_wire_params)

pytestmark = pytest.mark.gpu

WIRE = sta_wire_params(0.0021, 0.0017, 0.19, 0.23)


def _design(fanouts, seed):
    rng = np.random.default_rng(seed)
    fo = np.asarray(fanouts, np.int64)
    n_pins = int(len(fo) + fo.sum())
    perm = rng.permutation(n_pins).astype(np.int32)
    ptr = np.zeros(len(fo) + 1, np.int32)
    ptr[1:] = np.cumsum(fo)
    x = rng.uniform(0.0, 300.0, n_pins).astype(np.float32)
    y = rng.integers(0, 40, n_pins).astype(np.float32) * 2.5  # ties in y
    return SimpleNamespace(n_pins=n_pins, n_nets=len(fo), n_sinks=int(ptr[-1]), net_driver=perm[: len(fo)],
                           net_sink_ptr=ptr, net_sink_pin=perm[len(fo):], x=x, y=y)


def _estimate(d, noalloc):
    import torch
    dev = torch.device("cuda:0")

    def t(a, dt):
        return torch.as_tensor(np.ascontiguousarray(a, dt), device=dev)

    drv, ptr, pins = t(d.net_driver, np.int32), t(d.net_sink_ptr, np.int32), t(d.net_sink_pin, np.int32)
    x, y = t(d.x, np.float32), t(d.y, np.float32)
    g = sta_graph_desc(d.n_pins, 0, d.n_nets, 0, 0, None, None, None, None, None, drv.data_ptr(), ptr.data_ptr(),
                       pins.data_ptr(), STA_DEVICE)
    n_nodes = d.n_nets + 3 * d.n_sinks
    out = {"net_node_ptr": torch.full((d.n_nets + 1,), -7, dtype=torch.int64, device=dev),
           "parent": torch.full((max(n_nodes, 1),), -7, dtype=torch.int32, device=dev),
           "res_kohm": torch.full((max(n_nodes, 1),), -7.0, dtype=torch.float32, device=dev),
           "cap_ff": torch.full((max(n_nodes, 1),), -7.0, dtype=torch.float32, device=dev),
           "sink_node": torch.full((max(d.n_sinks, 1),), -7, dtype=torch.int32, device=dev)}
    stream = torch.cuda.current_stream(dev)
    args = (g, x, y, WIRE, out["net_node_ptr"], out["parent"], out["res_kohm"], out["cap_ff"], out["sink_node"])
    if noalloc:
        sta_estimate_rc_noalloc(*args, stream=stream)
    else:
        sta_estimate_rc(*args, mem=STA_DEVICE, stream=stream)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _same(a, b):
    for k in a:
        av, bv = a[k], b[k]
        if av.dtype == np.float32:
            av, bv = av.view(np.uint32), bv.view(np.uint32)
        bad = np.flatnonzero(av != bv)
        assert bad.size == 0, f"{k} differs at {bad[:8].tolist()}"


def test_noalloc_matches_allocating_estimator_twice():
    rng = np.random.default_rng(3)
    big = [5000, 700, 65, 100]                      # block tier (> 64 pins)
    mid = rng.integers(8, 64, 300).tolist()         # wave tier (9..64 pins)
    small = rng.integers(0, 8, 20000).tolist()      # lane tier (<= 8 pins)
    first = _design(big + mid + small, seed=1)
    print(f"[noalloc] first call: {first.n_nets} nets, {first.n_pins} pins", flush=True)
    _same(_estimate(first, True), _estimate(first, False))
    second = _design([80] + mid[:40] + small[:3000], seed=2)
    print(f"[noalloc] second call: {second.n_nets} nets, {second.n_pins} pins", flush=True)
    _same(_estimate(second, True), _estimate(second, False))


def test_noalloc_rejects_big_nets_beyond_its_scratch():
    """Nets of more than 64 pins holding more pins in all than the fixed
    scratch takes give STA_E_UNSUPPORTED before any tree is built; the entry
    point stays usable."""
    over = _design([12000] * 11, seed=4)  # 132,011 pins in nets above 64 pins
    with pytest.raises(StaError) as e:
        _estimate(over, True)
    assert e.value.status == STA_E_UNSUPPORTED
    ok = _design([3000, 70, 9, 3], seed=5)
    _same(_estimate(ok, True), _estimate(ok, False))
